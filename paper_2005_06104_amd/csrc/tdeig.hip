// Eigen-decomposition of a real symmetric tridiagonal matrix (n <= 512) by
// divide and conquer, bottom-up from leaves of size one:
//
//  * Cuppen's tear (Cuppen 1981): splitting T between rows m-1 and m with
//    coupling e gives T = diag(T1', T2') + e u u^T, u = e_{m-1} + e_m, where
//    T1', T2' have e subtracted from the two diagonal entries at the cut.
//    With T1' = Q1 L1 Q1^T and T2' = Q2 L2 Q2^T the merged problem is
//    diag(L1, L2) + e z z^T, z = (last row of Q1, first row of Q2).
//  * Deflation (Dongarra & Sorensen 1987): entries with |rho z_j| <= tol keep
//    (d_j, e_j); two poles closer than the tolerance are combined by a Givens
//    rotation that zeroes one z entry.
//  * The secular equation 1 + rho sum_j z_j^2 / (d_j - lambda) = 0 on each
//    interval between poles, solved for tau = lambda - d_o relative to the
//    nearer pole d_o (so that lambda - d_j is known to high relative
//    accuracy) by Newton steps on tau f(tau), safeguarded by bisection, until
//    f vanishes to within the rounding of its terms.
//  * Eigenvectors from the Loewner-type recomputation of z (Gu & Eisenstat
//    1995): zhat_j^2 = prod_i (lambda_i - d_j) / (rho prod_{i != j} (d_i - d_j)),
//    v_i = (zhat_j / (d_j - lambda_i))_j, normalised; numerically orthogonal
//    whatever the clustering of the roots.
//
// The size is padded to a power of two P with decoupled diagonal entries
// above the Gershgorin bound (their couplings are zero, so they deflate in
// every merge and end up as the top P - n eigenvalues).  The matrix is scaled
// by max(|D|, |E|) first.  The levels with nodes of up to 16 entries run in
// one launch (one workgroup per 16 leaves, in LDS); every larger level is
// five launches over all the nodes of the level: preparation (z, sort,
// deflation), secular roots, zhat and final order, eigenvector columns, and
// the block-diagonal product with the children's eigenvectors.  Nothing waits
// on another workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "wave.h"

namespace {

constexpr int DC_PREP_NT = 512;   // threads of the per-node preparation kernel
constexpr int DC_WNT = 256;       // four waves: one (node, index) pair each
constexpr int DC_PMAX = 512;
constexpr int DC_SECULAR_MAXIT = 200;
static_assert(DC_PREP_NT >= DC_PMAX, "the preparation kernel holds one entry per thread");

struct DcArgs {
  int P, s;                 // padded size, node size at this level
  const double* d;          // [P] children's eigenvalues (ascending per child)
  double* dnew;             // [P] the nodes' eigenvalues, ascending per node
  const double* E;          // [P] scaled couplings: E[m-1] joins rows m-1 and m
  const double* Zo;         // [P*P] row-major, children's eigenvectors (block diagonal)
  double* Zn;               // [P*P] the nodes' eigenvectors
  double* M;                // [P*P] node blocks: children's basis -> node eigenvectors
  int* perm;                // sorted position -> node-local index
  double* ds;               // sorted (sign-adjusted) poles after the deflation rotations
  int* ndinv;               // sorted position -> root index, -1 when deflated
  double* dk;               // [K] poles that take part in the secular equation
  double* zk;               // [K] their z entries
  int* nd;                  // [K] their sorted positions
  int* rp;                  // rotations: positions (rp, rq), cosine rc, sine rs
  int* rq;
  double* rc;
  double* rs;
  int* orig;                // [K] root i = dk[orig] + tau
  double* tau;
  double* zhat;
  int* colpos;              // sorted position -> final column (ascending eigenvalue)
  int* cnt;                 // per node: K, number of rotations
  double* par;              // per node: sign of the coupling, rho = 2 |coupling|
};

// Several independent tridiagonal problems (the charge blocks of one
// block-diagonal matrix) run side by side: every launch takes the arguments
// of up to DC_BMAX problems and finds its own in blockIdx.y (blockIdx.z for
// the tiled product); the grid is sized for the largest problem and the
// workgroups past a smaller problem's extent return at once.
constexpr int DC_BMAX = 16;
struct DcBatch {
  int n;            // problems in the launch
  int nodes_max;    // tiled product: z extent per problem
  DcArgs a[DC_BMAX];
};
struct DcInit {
  const double* D;
  const double* E;
  int n, P;
  double* d;
  double* Ep;
  double* Z;
  double* scale;
};
struct DcInitBatch {
  int n;
  DcInit b[DC_BMAX];
};
struct DcLeaf {
  double* dg;
  const double* E;
  double* Z;
  int P, S0;
};
struct DcLeafBatch {
  int n;
  DcLeaf b[DC_BMAX];
};
struct DcFinish {
  const double* d;
  const double* Z;
  const double* scale;
  int n, P;
  double* D;
  double* Zout;
};
struct DcFinishBatch {
  int n;
  DcFinish b[DC_BMAX];
};
// kernel arguments are limited to 4 KiB
static_assert(sizeof(DcBatch) <= 4096 && sizeof(DcInitBatch) <= 4096 && sizeof(DcLeafBatch) <= 4096 &&
                  sizeof(DcFinishBatch) <= 4096,
              "batched divide-and-conquer arguments too large");

// whole-wave reductions (every lane gets the result; all 64 lanes active)
__device__ inline double wave_sum(double v) { return wave::sum(v); }
__device__ inline double wave_prod(double v) { return wave::prod(v); }
__device__ inline double wave_max(double v) { return wave::max(v); }

// ---------------------------------------------------------------- set-up
// Scaled, torn, padded diagonal (the leaves' eigenvalues), couplings and
// Z = I.  Every workgroup finds the same scale (the same reduction order);
// workgroup 0 writes the vectors, all share the rows of Z.
__global__ __launch_bounds__(1024) void dc_init_kernel(const DcInitBatch bt) {
  if ((int)blockIdx.y >= bt.n) return;
  const DcInit ar = bt.b[blockIdx.y];
  const double* __restrict__ D = ar.D;
  const double* __restrict__ E = ar.E;
  const int n = ar.n, P = ar.P;
  double* __restrict__ d = ar.d;
  double* __restrict__ Ep = ar.Ep;
  double* __restrict__ Z = ar.Z;
  double* __restrict__ scale_out = ar.scale;
  __shared__ double red[2][16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double md = 0.0, me = 0.0;
  for (int i = tid; i < n; i += blockDim.x) md = fmax(md, fabs(D[i]));
  for (int i = tid; i < n - 1; i += blockDim.x) me = fmax(me, fabs(E[i]));
  md = wave_max(md);
  me = wave_max(me);
  if (lane == 0) {
    red[0][wave] = md;
    red[1][wave] = me;
  }
  __syncthreads();
  md = me = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    md = fmax(md, red[0][w]);
    me = fmax(me, red[1][w]);
  }
  double scale = fmax(md, me);
  if (!(scale > 0.0)) scale = 1.0;   // zero matrix (or NaN: caught by the caller's checks)
  const double inv = 1.0 / scale;
  const double bound = md * inv + 2.0 * me * inv;
  if (blockIdx.x == 0) {
    if (tid == 0) *scale_out = scale;
    for (int i = tid; i < P; i += blockDim.x) {
      const double e = i < n - 1 ? E[i] * inv : 0.0;
      const double em = (i >= 1 && i - 1 < n - 1) ? E[i - 1] * inv : 0.0;
      Ep[i] = e;
      // every m in [1, P) is a cut of exactly one level: subtract both couplings
      d[i] = i < n ? D[i] * inv - e - em : 2.0 * bound + 1.0;
    }
  }
  for (long long k = (long long)blockIdx.x * blockDim.x + tid; k < (long long)P * P;
       k += (long long)gridDim.x * blockDim.x)
    Z[k] = (k / P == k % P) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- level kernels
// Preparation, one workgroup per node: z, sign, sort by merging the two
// sorted children, deflation: small z entries in parallel, then one thread
// walks the remaining entries in sorted order (the pair tests precomputed,
// recomputed only after a rotation changed the left entry).
__global__ __launch_bounds__(DC_PREP_NT) void dc_prep_kernel(const DcBatch bt) {
  if ((int)blockIdx.y >= bt.n) return;
  const DcArgs a = bt.a[blockIdx.y];
  if ((int)blockIdx.x * a.s >= a.P) return;   // past this problem's nodes
  __shared__ double s_ds[DC_PMAX], s_zs[DC_PMAX];
  __shared__ int s_nd[DC_PMAX], s_inv[DC_PMAX];
  __shared__ double s_max[DC_PREP_NT / 64];
  __shared__ int s_lst[DC_PMAX], s_pd[DC_PMAX];
  __shared__ double s_pc[DC_PMAX], s_ps[DC_PMAX], s_pt[DC_PMAX];
  __shared__ int s_wcnt[DC_PREP_NT / 64];
  __shared__ int s_K;
  const int b = blockIdx.x, s = a.s, h = s / 2, P = a.P, tid = threadIdx.x;
  const int base = b * s;
  const double coupling = a.E[base + h - 1];
  const double sgn = coupling >= 0.0 ? 1.0 : -1.0;
  const double r = 2.0 * fabs(coupling);
  const double rs2 = 0.70710678118654752440;   // 1 / sqrt(2): |z| = sqrt(2) before scaling
  double lmax = 0.0;
  for (int j = tid; j < s; j += DC_PREP_NT) {
    const bool left = j < h;
    const double v = sgn * a.d[base + j];
    // position within the own child in ascending order of sgn * d
    const int jo = left ? j : j - h;
    const int po = sgn > 0.0 ? jo : h - 1 - jo;
    // elements of the other child that sort before: strictly smaller for a
    // left element, smaller or equal for a right element (ties: left first)
    const int ob = left ? base + h : base;
    int lo = 0, hi = h;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const int idx = sgn > 0.0 ? mid : h - 1 - mid;   // mid-th in ascending sgn order
      const double w = sgn * a.d[ob + idx];
      const bool before = left ? (w < v) : (w <= v);
      if (before) lo = mid + 1;
      else hi = mid;
    }
    const int rank = po + lo;
    const int zrow = left ? base + h - 1 : base + h;
    const double z = a.Zo[(size_t)zrow * P + base + j] * rs2;
    s_ds[rank] = v;
    s_zs[rank] = z;
    a.perm[base + rank] = j;
    lmax = fmax(lmax, fabs(v));
  }
  lmax = wave_max(lmax);
  const int lane = tid & 63, wv = tid >> 6;
  if (lane == 0) s_max[wv] = lmax;
  __syncthreads();
  double dm = 0.0;
  for (int w = 0; w < DC_PREP_NT / 64; ++w) dm = fmax(dm, s_max[w]);
  const double tol = 8.0 * 2.220446049250313e-16 * fmax(dm, r);
  // entries that keep a z component, compacted in sorted order (s <= the
  // number of threads: one entry each)
  const bool live = tid < s && r * fabs(s_zs[tid]) > tol;
  const unsigned long long bal = __ballot(live);
  if (lane == 0) s_wcnt[wv] = __popcll(bal);
  if (tid < s) s_inv[tid] = -1;
  __syncthreads();
  int off = 0, L = 0;
  for (int w = 0; w < DC_PREP_NT / 64; ++w) {
    if (w < wv) off += s_wcnt[w];
    L += s_wcnt[w];
  }
  if (live) s_lst[off + __popcll(bal & ((1ull << lane) - 1))] = tid;
  __syncthreads();
  // the test of each neighbouring pair with the values before any rotation;
  // it stands unless the left entry has just received a rotation
  if (tid + 1 < L) {
    const int p = s_lst[tid], q = s_lst[tid + 1];
    const double sv = s_zs[p], cv = s_zs[q];
    const double ta = hypot(cv, sv);
    const double c = cv / ta, sn = -sv / ta;
    s_pc[tid] = c;
    s_ps[tid] = sn;
    s_pt[tid] = ta;
    s_pd[tid] = fabs((s_ds[q] - s_ds[p]) * c * sn) <= tol ? 1 : 0;
  }
  __syncthreads();
  if (tid == 0) {
    int K = 0, m = 0;
    bool rotated = false;
    int pj = L > 0 ? s_lst[0] : -1;
    for (int k = 1; k < L; ++k) {
      const int j = s_lst[k];
      double c, sn, ta;
      bool defl;
      if (!rotated) {
        c = s_pc[k - 1];
        sn = s_ps[k - 1];
        ta = s_pt[k - 1];
        defl = s_pd[k - 1] != 0;
      } else {
        const double sv = s_zs[pj], cv = s_zs[j];
        ta = hypot(cv, sv);
        c = cv / ta;
        sn = -sv / ta;
        defl = fabs((s_ds[j] - s_ds[pj]) * c * sn) <= tol;
      }
      if (defl) {
        // rotate (pj, j): z_pj -> 0, z_j -> ta; pj keeps the mixed pole
        s_zs[j] = ta;
        s_zs[pj] = 0.0;
        a.rp[base + m] = pj;
        a.rq[base + m] = j;
        a.rc[base + m] = c;
        a.rs[base + m] = sn;
        ++m;
        const double dp = s_ds[pj], dj = s_ds[j];
        s_ds[pj] = dp * c * c + dj * sn * sn;
        s_ds[j] = dp * sn * sn + dj * c * c;
        rotated = true;
      } else {
        s_nd[K] = pj;
        s_inv[pj] = K;
        ++K;
        rotated = false;
      }
      pj = j;
    }
    if (pj >= 0) {
      s_nd[K] = pj;
      s_inv[pj] = K;
      ++K;
    }
    s_K = K;
    a.cnt[2 * b] = K;
    a.cnt[2 * b + 1] = m;
    a.par[2 * b] = sgn;
    a.par[2 * b + 1] = r;
  }
  __syncthreads();
  const int K = s_K;
  for (int j = tid; j < s; j += DC_PREP_NT) {
    a.ds[base + j] = s_ds[j];
    a.ndinv[base + j] = s_inv[j];
  }
  for (int i = tid; i < K; i += DC_PREP_NT) {
    const int p = s_nd[i];
    a.nd[base + i] = p;
    a.dk[base + i] = s_ds[p];
    a.zk[base + i] = s_zs[p];
  }
}

// Secular roots, one wave per (node, root i < K).
__global__ __launch_bounds__(DC_WNT) void dc_secular_kernel(const DcBatch bt) {
  if ((int)blockIdx.y >= bt.n) return;
  const DcArgs a = bt.a[blockIdx.y];
  const int gw = (blockIdx.x * DC_WNT + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  const int s = a.s;
  const int b = gw / s, i = gw % s;
  if (b * s >= a.P) return;
  const int K = a.cnt[2 * b];
  if (i >= K) return;
  const int base = b * s;
  const double r = a.par[2 * b + 1];
  const double* dk = a.dk + base;
  const double* zk = a.zk + base;
  constexpr int PL = DC_PMAX / 64;
  double dj[PL], z2[PL];
  double zsum = 0.0;
#pragma unroll
  for (int t = 0; t < PL; ++t) {
    const int j = lane + 64 * t;
    dj[t] = j < K ? dk[j] : 1e300;   // padding lanes: zero weight far from every pole
    z2[t] = j < K ? zk[j] * zk[j] : 0.0;
    zsum += z2[t];
  }
  zsum = wave_sum(zsum);
  const bool last = i + 1 == K;
  const double lo_abs = dk[i];
  const double hi_abs = last ? dk[i] + r * zsum : dk[i + 1];
  const double mid = 0.5 * (lo_abs + hi_abs);
  double fm = 0.0;
#pragma unroll
  for (int t = 0; t < PL; ++t) fm += z2[t] / (dj[t] - mid);
  fm = 1.0 + r * wave_sum(fm);
  const int o = (!last && fm <= 0.0) ? i + 1 : i;
  const double dorg = dk[o];
#pragma unroll
  for (int t = 0; t < PL; ++t) dj[t] -= dorg;   // delta_j = d_j - d_o
  double lo, hi;
  if (o == i) {
    lo = 0.0;
    hi = last ? r * zsum : mid - dorg;
  } else {
    lo = mid - dorg;
    hi = 0.0;
  }
  double tau = 0.5 * (lo + hi);
  for (int it = 0; it < DC_SECULAR_MAXIT; ++it) {
    double f = 0.0, fp = 0.0, fa = 0.0;
#pragma unroll
    for (int t = 0; t < PL; ++t) {
      const double q = 1.0 / (dj[t] - tau);
      const double tt = z2[t] * q;
      f += tt;
      fp += tt * q;
      fa += fabs(tt);
    }
    f = 1.0 + r * wave_sum(f);
    fp = r * wave_sum(fp);
    fa = 1.0 + r * wave_sum(fa);
    // f vanishes to within the rounding of its terms
    if (fabs(f) <= 8.0 * 2.220446049250313e-16 * fa) break;
    if (f > 0.0) hi = tau;
    else lo = tau;
    if (hi - lo <= 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi))) break;
    // Newton step on tau f(tau), which has no pole at the origin
    double tn = tau - tau * f / (f + tau * fp);
    if (!(isfinite(tn) && tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (fabs(tn - tau) <= 2.0 * 2.220446049250313e-16 * fabs(tau)) {
      tau = tn;
      break;
    }
    tau = tn;
  }
  if (lane == 0) {
    a.orig[base + i] = o;
    a.tau[base + i] = tau;
  }
}

// zhat_j (j < K) and the final column of sorted position j (all j < s), one
// wave per (node, j).
__global__ __launch_bounds__(DC_WNT) void dc_zhat_kernel(const DcBatch bt) {
  if ((int)blockIdx.y >= bt.n) return;
  const DcArgs a = bt.a[blockIdx.y];
  const int gw = (blockIdx.x * DC_WNT + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  const int s = a.s;
  const int b = gw / s, j = gw % s;
  if (b * s >= a.P) return;
  const int base = b * s;
  const int K = a.cnt[2 * b];
  const double sgn = a.par[2 * b], r = a.par[2 * b + 1];
  const double* dk = a.dk + base;
  if (j < K) {
    const double dj = dk[j];
    double p = 1.0;
    for (int i = lane; i < K; i += 64) {
      const double num = (dk[a.orig[base + i]] - dj) + a.tau[base + i];
      p *= i == j ? num / r : num / (dk[i] - dj);
    }
    p = wave_prod(p);
    if (lane == 0) a.zhat[base + j] = copysign(sqrt(fabs(p)), a.zk[base + j]);
  }
  // eigenvalue at sorted position q (sign restored); rank among the node's
  auto value = [&](int q) {
    const int ri = a.ndinv[base + q];
    const double l = ri >= 0 ? dk[a.orig[base + ri]] + a.tau[base + ri] : a.ds[base + q];
    return sgn * l;
  };
  const double vj = value(j);
  int c = 0;
  for (int q = lane; q < s; q += 64) {
    const double vq = value(q);
    c += (vq < vj || (vq == vj && q < j)) ? 1 : 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (lane == 0) {
    a.colpos[base + j] = c;
    a.dnew[base + c] = vj;
  }
}

// Column of the node's eigenvector matrix for sorted position p, one wave per
// (node, p): the secular eigenvector (or e_p when deflated) in the sorted
// basis, the deflation rotations undone in reverse order, rows returned to the
// children's order, stored at the final column.
__global__ __launch_bounds__(DC_WNT) void dc_vectors_kernel(const DcBatch bt) {
  if ((int)blockIdx.y >= bt.n) return;
  const DcArgs a = bt.a[blockIdx.y];
  __shared__ double sy[DC_WNT / 64][DC_PMAX];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gw = (blockIdx.x * DC_WNT + threadIdx.x) >> 6;
  const int s = a.s, P = a.P;
  const int b = gw / s, p = gw % s;
  if (b * s >= P) return;
  const int base = b * s;
  double* y = sy[wv];
  for (int q = lane; q < s; q += 64) y[q] = 0.0;
  const int ri = a.ndinv[base + p];
  if (ri < 0) {
    if (lane == 0) y[p] = 1.0;
  } else {
    const int K = a.cnt[2 * b];
    const double* dk = a.dk + base;
    const double dorg = dk[a.orig[base + ri]], ta = a.tau[base + ri];
    double nrm = 0.0;
    for (int j = lane; j < K; j += 64) {
      const double v = a.zhat[base + j] / ((dk[j] - dorg) - ta);
      y[a.nd[base + j]] = v;
      nrm += v * v;
    }
    nrm = wave_sum(nrm);
    const double inv = 1.0 / sqrt(nrm);
    for (int j = lane; j < K; j += 64) y[a.nd[base + j]] *= inv;
  }
  // lane 0 reads what the other lanes of the wave stored
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int m = a.cnt[2 * b + 1];
  if (lane == 0) {
    for (int t = m - 1; t >= 0; --t) {
      const int pp = a.rp[base + t], qq = a.rq[base + t];
      const double c = a.rc[base + t], sn = a.rs[base + t];
      const double yp = y[pp], yq = y[qq];
      y[pp] = c * yp - sn * yq;
      y[qq] = sn * yp + c * yq;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int col = a.colpos[base + p];
  for (int q = lane; q < s; q += 64) a.M[(size_t)(base + a.perm[base + q]) * P + base + col] = y[q];
}

// Zn[node] = blockdiag(Z1, Z2) M[node]: rows of the left child combine the
// first s/2 rows of M, rows of the right child the last s/2.  Small nodes:
// one thread per output entry.
__global__ __launch_bounds__(256) void dc_gemm_small_kernel(const DcBatch bt) {
  if ((int)blockIdx.y >= bt.n) return;
  const DcArgs a = bt.a[blockIdx.y];
  const int s = a.s, h = s / 2, P = a.P;
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)P * s) return;
  const int row = (int)(idx / s), cl = (int)(idx % s);
  const int base = row / s * s;
  const int k0 = base + ((row - base) < h ? 0 : h);
  const double* zr = a.Zo + (size_t)row * P;
  double acc = 0.0;
  for (int k = k0; k < k0 + h; ++k) acc += zr[k] * a.M[(size_t)k * P + base + cl];
  a.Zn[(size_t)row * P + base + cl] = acc;
}

// Nodes of 64 and more: 32 x 32 output tiles, 256 threads of 2 x 2 entries,
// k in chunks of 32 through LDS.
__global__ __launch_bounds__(256) void dc_gemm_tiled_kernel(const DcBatch bt) {
  __shared__ double sa[32][33], sb[32][33];
  // blockIdx.z = node + nodes_max * problem
  const int pb = (int)blockIdx.z / bt.nodes_max;
  if (pb >= bt.n) return;
  const DcArgs a = bt.a[pb];
  const int s = a.s, h = s / 2, P = a.P;
  const int tiles = s / 32;
  const int b = (int)blockIdx.z % bt.nodes_max, ti = blockIdx.y, tj = blockIdx.x;
  if (ti >= tiles || tj >= tiles || b * s >= P) return;
  const int base = b * s;
  const int r0 = base + ti * 32, c0 = base + tj * 32;
  const int k0 = base + (ti * 32 < h ? 0 : h);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int kc = k0; kc < k0 + h; kc += 32) {
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
      const int rr = e >> 5, cc = e & 31;
      sa[rr][cc] = a.Zo[(size_t)(r0 + rr) * P + kc + cc];
      sb[rr][cc] = a.M[(size_t)(kc + rr) * P + c0 + cc];
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
      const double a0 = sa[ty][k], a1 = sa[ty + 16][k];
      const double b0 = sb[k][tx], b1 = sb[k][tx + 16];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
  a.Zn[(size_t)(r0 + ty) * P + c0 + tx] = acc[0][0];
  a.Zn[(size_t)(r0 + ty) * P + c0 + tx + 16] = acc[0][1];
  a.Zn[(size_t)(r0 + ty + 16) * P + c0 + tx] = acc[1][0];
  a.Zn[(size_t)(r0 + ty + 16) * P + c0 + tx + 16] = acc[1][1];
}

// D[j] = scale d[j], Zout (column-major n x n) = leading block of Z.
__global__ void dc_finish_kernel(const DcFinishBatch bt) {
  if ((int)blockIdx.y >= bt.n) return;
  const DcFinish ar = bt.b[blockIdx.y];
  const double* __restrict__ d = ar.d;
  const double* __restrict__ Z = ar.Z;
  const double* __restrict__ scale = ar.scale;
  const int n = ar.n, P = ar.P;
  double* __restrict__ D = ar.D;
  double* __restrict__ Zout = ar.Zout;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) D[idx] = d[idx] * *scale;
  if (idx >= (long long)n * n) return;
  const int j = (int)(idx / n), m = (int)(idx % n);
  Zout[idx] = Z[(size_t)m * P + j];
}

// ---------------------------------------------------------------- small levels
// Levels with nodes of 2 .. DC_LEAF entries, all in one launch: one workgroup
// per block of DC_LEAF leaves, everything in LDS, one thread per entry, root or
// node (the same steps as the level kernels, with the sums over a node's at
// most DC_LEAF poles taken serially by one thread).  On return d holds each
// block's eigenvalues (ascending) and Z its diagonal block of eigenvectors
// (the rest of Z is the identity's zeros).
constexpr int DC_LEAF = 16;
constexpr int DC_LNT = 256;
static_assert(DC_LNT >= DC_LEAF * 2, "leaf kernel thread count");

__global__ __launch_bounds__(DC_LNT) void dc_leaf_kernel(const DcLeafBatch bt) {
  if ((int)blockIdx.y >= bt.n) return;
  const DcLeaf ar = bt.b[blockIdx.y];
  double* __restrict__ dg = ar.dg;
  const double* __restrict__ E = ar.E;
  double* __restrict__ Z = ar.Z;
  const int P = ar.P, S0 = ar.S0;
  if ((int)blockIdx.x * S0 >= P) return;   // past this problem's leaves
  __shared__ double sZ[DC_LEAF][DC_LEAF + 1], sZn[DC_LEAF][DC_LEAF + 1], sM[DC_LEAF][DC_LEAF + 1];
  __shared__ double sY[DC_LEAF][DC_LEAF + 1];
  __shared__ double sd[DC_LEAF], sdn[DC_LEAF], s_ds[DC_LEAF], s_zs[DC_LEAF], s_dk[DC_LEAF], s_zk[DC_LEAF];
  __shared__ double s_rc[DC_LEAF], s_rs[DC_LEAF], s_tau[DC_LEAF], s_zhat[DC_LEAF];
  __shared__ int s_perm[DC_LEAF], s_inv[DC_LEAF], s_nd[DC_LEAF], s_rp[DC_LEAF], s_rq[DC_LEAF], s_orig[DC_LEAF];
  __shared__ int s_col[DC_LEAF];
  __shared__ int s_K[DC_LEAF], s_m[DC_LEAF];
  __shared__ double s_sgn[DC_LEAF], s_r[DC_LEAF];
  const int tid = threadIdx.x, g0 = blockIdx.x * S0;
  constexpr double EPS = 2.220446049250313e-16;
  for (int e = tid; e < S0 * S0; e += DC_LNT) sZ[e / S0][e % S0] = (e / S0 == e % S0) ? 1.0 : 0.0;
  for (int j = tid; j < S0; j += DC_LNT) sd[j] = dg[g0 + j];
  __syncthreads();
  for (int s = 2; s <= S0; s *= 2) {
    const int h = s / 2, nn = S0 / s;
    // ---- node constants; merge the two sorted children; z
    if (tid < nn) {
      const double coupling = E[g0 + tid * s + h - 1];
      s_sgn[tid] = coupling >= 0.0 ? 1.0 : -1.0;
      s_r[tid] = 2.0 * fabs(coupling);
    }
    __syncthreads();
    if (tid < S0) {
      const int b = tid / s, j = tid % s, base = b * s;
      const double sgn = s_sgn[b];
      const bool left = j < h;
      const double v = sgn * sd[base + j];
      const int jo = left ? j : j - h;
      const int po = sgn > 0.0 ? jo : h - 1 - jo;
      const int ob = left ? base + h : base;
      int lo = 0, hi = h;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int idx = sgn > 0.0 ? mid : h - 1 - mid;
        const double w = sgn * sd[ob + idx];
        const bool before = left ? (w < v) : (w <= v);
        if (before) lo = mid + 1;
        else hi = mid;
      }
      const int rank = po + lo;
      const int zrow = left ? base + h - 1 : base + h;
      s_ds[base + rank] = v;
      s_zs[base + rank] = sZ[zrow][base + j] * 0.70710678118654752440;
      s_perm[base + rank] = j;
      s_inv[base + rank] = -1;
    }
    __syncthreads();
    // ---- deflation, one thread per node (at most DC_LEAF entries)
    if (tid < nn) {
      const int base = tid * s;
      const double r = s_r[tid];
      double dm = 0.0;
      for (int j = 0; j < s; ++j) dm = fmax(dm, fabs(s_ds[base + j]));
      const double tol = 8.0 * EPS * fmax(dm, r);
      int K = 0, m = 0, pj = -1;
      for (int j = 0; j < s; ++j) {
        if (!(r * fabs(s_zs[base + j]) > tol)) continue;   // z entry deflated
        if (pj < 0) {
          pj = j;
          continue;
        }
        const double sv = s_zs[base + pj], cv = s_zs[base + j];
        const double ta = hypot(cv, sv);
        const double c = cv / ta, sn = -sv / ta;
        if (fabs((s_ds[base + j] - s_ds[base + pj]) * c * sn) <= tol) {
          s_zs[base + j] = ta;
          s_zs[base + pj] = 0.0;
          s_rp[base + m] = pj;
          s_rq[base + m] = j;
          s_rc[base + m] = c;
          s_rs[base + m] = sn;
          ++m;
          const double dp = s_ds[base + pj], dj = s_ds[base + j];
          s_ds[base + pj] = dp * c * c + dj * sn * sn;
          s_ds[base + j] = dp * sn * sn + dj * c * c;
        } else {
          s_nd[base + K] = pj;
          s_inv[base + pj] = K;
          ++K;
        }
        pj = j;
      }
      if (pj >= 0) {
        s_nd[base + K] = pj;
        s_inv[base + pj] = K;
        ++K;
      }
      for (int i = 0; i < K; ++i) {
        s_dk[base + i] = s_ds[base + s_nd[base + i]];
        s_zk[base + i] = s_zs[base + s_nd[base + i]];
      }
      s_K[tid] = K;
      s_m[tid] = m;
    }
    __syncthreads();
    // ---- secular roots, one thread per (node, root)
    if (tid < S0) {
      const int b = tid / s, i = tid % s, base = b * s;
      const int K = s_K[b];
      if (i < K) {
        const double r = s_r[b];
        const double* dk = s_dk + base;
        const double* zk = s_zk + base;
        double zsum = 0.0;
        for (int j = 0; j < K; ++j) zsum += zk[j] * zk[j];
        const bool last = i + 1 == K;
        const double lo_abs = dk[i];
        const double hi_abs = last ? dk[i] + r * zsum : dk[i + 1];
        const double mid = 0.5 * (lo_abs + hi_abs);
        double fm = 0.0;
        for (int j = 0; j < K; ++j) fm += zk[j] * zk[j] / (dk[j] - mid);
        fm = 1.0 + r * fm;
        const int o = (!last && fm <= 0.0) ? i + 1 : i;
        const double dorg = dk[o];
        double lo, hi;
        if (o == i) {
          lo = 0.0;
          hi = last ? r * zsum : mid - dorg;
        } else {
          lo = mid - dorg;
          hi = 0.0;
        }
        double tau = 0.5 * (lo + hi);
        for (int it = 0; it < DC_SECULAR_MAXIT; ++it) {
          double f = 0.0, fp = 0.0, fa = 0.0;
          for (int j = 0; j < K; ++j) {
            const double q = 1.0 / ((dk[j] - dorg) - tau);
            const double tt = zk[j] * zk[j] * q;
            f += tt;
            fp += tt * q;
            fa += fabs(tt);
          }
          f = 1.0 + r * f;
          fp = r * fp;
          fa = 1.0 + r * fa;
          if (fabs(f) <= 8.0 * EPS * fa) break;
          if (f > 0.0) hi = tau;
          else lo = tau;
          if (hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi))) break;
          double tn = tau - tau * f / (f + tau * fp);
          if (!(isfinite(tn) && tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
          if (fabs(tn - tau) <= 2.0 * EPS * fabs(tau)) {
            tau = tn;
            break;
          }
          tau = tn;
        }
        s_orig[base + i] = o;
        s_tau[base + i] = tau;
      }
    }
    __syncthreads();
    // ---- zhat_j (j < K) and the final column of every sorted position
    if (tid < S0) {
      const int b = tid / s, j = tid % s, base = b * s;
      const int K = s_K[b];
      const double sgn = s_sgn[b], r = s_r[b];
      const double* dk = s_dk + base;
      if (j < K) {
        const double dj = dk[j];
        double p = 1.0;
        for (int i = 0; i < K; ++i) {
          const double num = (dk[s_orig[base + i]] - dj) + s_tau[base + i];
          p *= i == j ? num / r : num / (dk[i] - dj);
        }
        s_zhat[base + j] = copysign(sqrt(fabs(p)), s_zk[base + j]);
      }
      auto value = [&](int q) {
        const int ri = s_inv[base + q];
        const double l = ri >= 0 ? dk[s_orig[base + ri]] + s_tau[base + ri] : s_ds[base + q];
        return sgn * l;
      };
      const double vj = value(j);
      int c = 0;
      for (int q = 0; q < s; ++q) {
        const double vq = value(q);
        c += (vq < vj || (vq == vj && q < j)) ? 1 : 0;
      }
      s_col[base + j] = c;
      sdn[base + c] = vj;
    }
    __syncthreads();
    // ---- eigenvector columns (rotations undone), scattered into the node block of M
    if (tid < S0) {
      const int b = tid / s, p = tid % s, base = b * s;
      double* y = sY[tid];
      for (int q = 0; q < s; ++q) y[q] = 0.0;
      const int ri = s_inv[base + p];
      if (ri < 0) {
        y[p] = 1.0;
      } else {
        const int K = s_K[b];
        const double* dk = s_dk + base;
        const double dorg = dk[s_orig[base + ri]], ta = s_tau[base + ri];
        double nrm = 0.0;
        for (int j = 0; j < K; ++j) {
          const double v = s_zhat[base + j] / ((dk[j] - dorg) - ta);
          y[s_nd[base + j]] = v;
          nrm += v * v;
        }
        const double inv = 1.0 / sqrt(nrm);
        for (int j = 0; j < K; ++j) y[s_nd[base + j]] *= inv;
      }
      for (int t = s_m[b] - 1; t >= 0; --t) {
        const int pp = s_rp[base + t], qq = s_rq[base + t];
        const double c = s_rc[base + t], sn = s_rs[base + t];
        const double yp = y[pp], yq = y[qq];
        y[pp] = c * yp - sn * yq;
        y[qq] = sn * yp + c * yq;
      }
      const int col = s_col[base + p];
      for (int q = 0; q < s; ++q) sM[base + s_perm[base + q]][base + col] = y[q];
    }
    __syncthreads();
    // ---- Zn = blockdiag(children) M on each node block
    for (int e = tid; e < S0 * s; e += DC_LNT) {
      const int row = e / s, cl = e % s;
      const int base = row / s * s;
      const int k0 = base + ((row - base) < h ? 0 : h);
      double acc = 0.0;
      for (int k = k0; k < k0 + h; ++k) acc += sZ[row][k] * sM[k][base + cl];
      sZn[row][base + cl] = acc;
    }
    __syncthreads();
    for (int e = tid; e < S0 * S0; e += DC_LNT) {
      const int row = e / S0, cl = e % S0;
      if (row / s == cl / s) sZ[row][cl] = sZn[row][cl];
    }
    for (int j = tid; j < S0; j += DC_LNT) sd[j] = sdn[j];
    __syncthreads();
  }
  for (int j = tid; j < S0; j += DC_LNT) dg[g0 + j] = sd[j];
  for (int e = tid; e < S0 * S0; e += DC_LNT) Z[(size_t)(g0 + e / S0) * P + g0 + e % S0] = sZ[e / S0][e % S0];
}

int dc_pad(int n) {
  int P = 1;
  while (P < n) P *= 2;
  return P;
}

}  // namespace

namespace kern {

size_t tridiag_eig_scratch_bytes(int n) {
  if (n < 1 || n > DC_PMAX) return 0;
  const size_t P = (size_t)dc_pad(n);
  // Z0, Z1, M; 12 double and 9 int arrays of P; per-node 2 int + 2 double; scale
  return sizeof(double) * (3 * P * P + 14 * P + 8) + sizeof(int) * (11 * P) + 32 * 256;
}

namespace {

// one problem's buffers, carved out of its scratch
struct DcPlan {
  int n = 0, P = 0, S0 = 0;
  double* D = nullptr;
  const double* E = nullptr;
  double* Zout = nullptr;
  double *Z0 = nullptr, *Z1 = nullptr, *dA = nullptr, *dB = nullptr, *Ep = nullptr, *scale = nullptr;
  DcArgs a{};   // the level-independent fields
  // current and next eigenvalue / eigenvector buffers (swapped per level)
  double *dc = nullptr, *dn = nullptr, *zc = nullptr, *zn = nullptr;
};

DcPlan dc_plan(double* D, const double* E, int n, double* Z, void* scratch) {
  DcPlan q;
  q.n = n;
  q.P = dc_pad(n);
  q.S0 = std::min(DC_LEAF, q.P);
  q.D = D;
  q.E = E;
  q.Zout = Z;
  const int P = q.P;
  char* p = static_cast<char*>(scratch);
  auto take_d = [&](size_t count) {
    double* r = reinterpret_cast<double*>(p);
    p += (count * sizeof(double) + 255) / 256 * 256;
    return r;
  };
  auto take_i = [&](size_t count) {
    int* r = reinterpret_cast<int*>(p);
    p += (count * sizeof(int) + 255) / 256 * 256;
    return r;
  };
  const size_t PP = (size_t)P * P;
  q.Z0 = take_d(PP);
  q.Z1 = take_d(PP);
  DcArgs& a = q.a;
  a.P = P;
  a.M = take_d(PP);
  q.dA = take_d(P);
  q.dB = take_d(P);
  q.Ep = take_d(P);
  a.ds = take_d(P);
  a.dk = take_d(P);
  a.zk = take_d(P);
  a.rc = take_d(P);
  a.rs = take_d(P);
  a.tau = take_d(P);
  a.zhat = take_d(P);
  a.par = take_d(2 * (size_t)P);
  q.scale = take_d(8);
  a.perm = take_i(P);
  a.ndinv = take_i(P);
  a.nd = take_i(P);
  a.rp = take_i(P);
  a.rq = take_i(P);
  a.orig = take_i(P);
  a.colpos = take_i(P);
  a.cnt = take_i(2 * (size_t)P);
  a.E = q.Ep;
  q.zc = q.Z0;
  q.zn = q.Z1;
  q.dc = q.dA;
  q.dn = q.dB;
  return q;
}

// up to DC_BMAX problems side by side
void dc_run_group(hipStream_t st, std::vector<DcPlan>& pl) {
  const int nb = (int)pl.size();
  // set-up: scaled, torn, padded diagonals and Z = I
  DcInitBatch ib{};
  ib.n = nb;
  int init_x = 1;
  for (int j = 0; j < nb; ++j) {
    const DcPlan& q = pl[j];
    ib.b[j] = DcInit{q.D, q.E, q.n, q.P, q.dA, q.Ep, q.Z0, q.scale};
    init_x = std::max(init_x, std::max(1, std::min(64, q.P * q.P / 4096)));
  }
  hipLaunchKernelGGL(dc_init_kernel, dim3(init_x, nb), dim3(1024), 0, st, ib);
  // the levels of up to DC_LEAF entries in one launch
  DcLeafBatch lb{};
  int leaf_x = 0;
  for (const DcPlan& q : pl) {
    if (q.P < 2) continue;
    lb.b[lb.n++] = DcLeaf{q.dA, q.Ep, q.Z0, q.P, q.S0};
    leaf_x = std::max(leaf_x, q.P / q.S0);
  }
  if (lb.n > 0) hipLaunchKernelGGL(dc_leaf_kernel, dim3(leaf_x, lb.n), dim3(DC_LNT), 0, st, lb);
  // larger levels: the problems whose padded size reaches s, in lock step
  int maxP = 0;
  for (const DcPlan& q : pl) maxP = std::max(maxP, q.P);
  for (int s = 2 * DC_LEAF; s <= maxP; s *= 2) {
    DcBatch bt{};
    std::vector<int> act;
    int pmax = 0;
    for (int j = 0; j < nb; ++j) {
      DcPlan& q = pl[j];
      if (q.S0 != DC_LEAF || q.P < s) continue;
      DcArgs a = q.a;
      a.s = s;
      a.d = q.dc;
      a.dnew = q.dn;
      a.Zo = q.zc;
      a.Zn = q.zn;
      bt.a[bt.n++] = a;
      act.push_back(j);
      pmax = std::max(pmax, q.P);
    }
    if (bt.n == 0) continue;
    const int nodes_max = pmax / s;
    bt.nodes_max = nodes_max;
    const int wblocks = (pmax * 64 + DC_WNT - 1) / DC_WNT;   // one wave per index of every node
    hipLaunchKernelGGL(dc_prep_kernel, dim3(nodes_max, bt.n), dim3(DC_PREP_NT), 0, st, bt);
    hipLaunchKernelGGL(dc_secular_kernel, dim3(wblocks, bt.n), dim3(DC_WNT), 0, st, bt);
    hipLaunchKernelGGL(dc_zhat_kernel, dim3(wblocks, bt.n), dim3(DC_WNT), 0, st, bt);
    hipLaunchKernelGGL(dc_vectors_kernel, dim3(wblocks, bt.n), dim3(DC_WNT), 0, st, bt);
    if (s < 64) {
      const long long tot = (long long)pmax * s;
      hipLaunchKernelGGL(dc_gemm_small_kernel, dim3((unsigned)((tot + 255) / 256), bt.n), dim3(256), 0, st, bt);
    } else {
      hipLaunchKernelGGL(dc_gemm_tiled_kernel, dim3(s / 32, s / 32, nodes_max * bt.n), dim3(256), 0, st, bt);
    }
    for (int j : act) {
      std::swap(pl[j].zc, pl[j].zn);
      std::swap(pl[j].dc, pl[j].dn);
    }
  }
  // eigenvalues unscaled, eigenvectors column-major
  DcFinishBatch fb{};
  fb.n = nb;
  long long fmax = 1;
  for (int j = 0; j < nb; ++j) {
    const DcPlan& q = pl[j];
    fb.b[j] = DcFinish{q.dc, q.zc, q.scale, q.n, q.P, q.D, q.Zout};
    fmax = std::max(fmax, std::max<long long>((long long)q.n * q.n, q.n));
  }
  hipLaunchKernelGGL(dc_finish_kernel, dim3((unsigned)((fmax + 255) / 256), nb), dim3(256), 0, st, fb);
}

}  // namespace

hipError_t tridiag_eig_batched(hipStream_t st, const TdEigJob* jobs, int n_jobs) {
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return hipErrorInvalidValue;
  for (int j = 0; j < n_jobs; ++j)
    if (jobs[j].n < 1 || jobs[j].n > DC_PMAX || !jobs[j].scratch) return hipErrorInvalidValue;
  for (int g = 0; g < n_jobs; g += DC_BMAX) {
    std::vector<DcPlan> pl;
    for (int j = g; j < std::min(n_jobs, g + DC_BMAX); ++j)
      pl.push_back(dc_plan(jobs[j].D, jobs[j].E, jobs[j].n, jobs[j].Z, jobs[j].scratch));
    dc_run_group(st, pl);
  }
  return hipGetLastError();
}

hipError_t tridiag_eig(hipStream_t st, double* D, const double* E, int n, double* Z, void* scratch) {
  const TdEigJob job{D, E, n, Z, scratch};
  return tridiag_eig_batched(st, &job, 1);
}

}  // namespace kern
