// Hermitian eigendecomposition for the mid-size Gram and density matrices of
// the method (n <= 1024; above 512 with the Q rows outside LDS): Householder reduction to real tridiagonal form by one
// cooperative launch, the tridiagonal eigenproblem by divide and conquer
// (tdeig.hip; rocSOLVER's on request), and one MFMA GEMM for the back
// transformation.
//
// The reduction is the unblocked Householder algorithm (Golub & Van Loan,
// Matrix Computations, Sec. 8.3.1; the LAPACK xHETD2 scheme with lower
// storage): for k = 0..n-2 the reflector H_k = I - tau v v^H with v_{k+1} = 1
// maps A[k+1:, k] to (beta, 0, ..., 0) with beta real, and the trailing block
// becomes H_k^H A H_k = A - v w^H - w v^H with x = tau A v,
// w = x - (tau/2)(x^H v) v.  Q = H_0 H_1 ... H_{n-2} is accumulated row by row.
//
// A library call per column costs a few microseconds of dispatch on this GPU,
// so the whole reduction is one launch: G workgroups keep the matrix rows
// (row r on workgroup r % G) and the matching rows of Q in LDS and exchange
// per column the vector x = tau A v and the next pivot row; every workgroup
// then forms x^H v from the whole x itself (no exchange of partial sums,
// whose publication after the row products was the last arrival).
// The exchange needs no barrier: every published complex is stored as four
// 64-bit words, each holding 32 bits of the value and the column's tag, and
// a reader polls the words it needs until all carry the current tag (one
// memory round trip instead of a flag round trip followed by the data).
// Every wait is bounded; a wait that runs out raises an error flag that
// makes every workgroup leave, and the caller then uses another solver.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "wave.h"

namespace {

constexpr int TNT = 256;            // threads per workgroup
constexpr int TD_LDS = 8192;        // complex128 slots for the A and Q rows (128 KiB)
constexpr int TD_NMAX = 512;
// Larger matrices (512 < n <= 1024): four rows per workgroup, up to 256
// workgroups (one per CU); the A rows stay in LDS (64 KiB) and the Q rows of
// the workgroup are accumulated in place in the output (each row read and
// written only by the threads that own it, from L2).
constexpr int TD_LDS_BIG = 4096;
constexpr int TD_NMAX_BIG = 1024;
constexpr int TD_G_BIG = 256;
constexpr int TD_ROWS = 128;        // rows per workgroup at most
constexpr unsigned SPIN_LIMIT = 1u << 22;

struct TdArgs {
  const double2* H;   // n x n Hermitian, row-major
  double2* Q;         // n x n out, row-major
  double* D;          // n out
  double* E;          // n-1 out
  // tagged words (four per complex, zero at launch), two buffers each:
  unsigned long long* xv;     // published x = tau A v, 2 x n
  unsigned long long* prow;   // published pivot row, 2 x n
  int* err;                   // 0 at launch; 1 when a wait ran out
  int n, G, R;
};

// Several independent matrices in one launch: sector s owns workgroups
// wg0[s] .. wg0[s+1] - 1 and its own exchange buffers, so the sectors (the
// charge blocks of a block-diagonal matrix) are reduced side by side.
constexpr int TD_MAXSEC = 16;
struct TdBatch {
  TdArgs sec[TD_MAXSEC];
  int wg0[TD_MAXSEC + 1];
  int nsec;
};

__device__ inline double2 cmul(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return double2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

__device__ inline double2 wave_sum(double2 v) { return double2{wave::sum(v.x), wave::sum(v.y)}; }

// Publish v under tag t: the low and high halves of both parts, each with
// the tag in the upper 32 bits of its word.
__device__ inline void put_tagged(unsigned long long* w, double2 v, unsigned t) {
  const unsigned long long tag = (unsigned long long)t << 32;
  const unsigned long long bx = (unsigned long long)__double_as_longlong(v.x);
  const unsigned long long by = (unsigned long long)__double_as_longlong(v.y);
  __hip_atomic_store(w + 0, tag | (bx & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 1, tag | (bx >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 2, tag | (by & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 3, tag | (by >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Read a value published under tag t; false (v untouched) while any of its
// words still holds an older tag.
__device__ inline bool get_tagged(const unsigned long long* w, unsigned t, double2* v) {
  const unsigned long long w0 = __hip_atomic_load(w + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long w1 = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long w2 = __hip_atomic_load(w + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long w3 = __hip_atomic_load(w + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((unsigned)(w0 >> 32) != t || (unsigned)(w1 >> 32) != t || (unsigned)(w2 >> 32) != t ||
      (unsigned)(w3 >> 32) != t)
    return false;
  v->x = __longlong_as_double((long long)(((w1 & 0xffffffffull) << 32) | (w0 & 0xffffffffull)));
  v->y = __longlong_as_double((long long)(((w3 & 0xffffffffull) << 32) | (w2 & 0xffffffffull)));
  return true;
}

// Reflector of column k from the pivot row: alpha = conj(row[k+1]),
// x = conj(row[k+2:]) with |x|^2 = xn2.  Every thread of every workgroup
// evaluates it with the same operands in the same order, so all agree bit
// for bit.  tau = sc = 0 (H_k = I) when the column is already reduced.
struct Reflector {
  double2 tau, sc;
  double beta;
};
__device__ inline Reflector reflector(double2 row_k1, double xn2) {
  const double2 al{row_k1.x, -row_k1.y};
  Reflector r;
  if (xn2 == 0.0 && al.y == 0.0) {
    r.beta = al.x;
    r.tau = r.sc = double2{0.0, 0.0};
  } else {
    const double nrm = sqrt(al.x * al.x + al.y * al.y + xn2);
    r.beta = al.x >= 0.0 ? -nrm : nrm;
    r.tau = double2{(r.beta - al.x) / r.beta, -al.y / r.beta};
    const double dr = al.x - r.beta, di = al.y;   // sc = 1 / (alpha - beta)
    const double den = dr * dr + di * di;
    r.sc = double2{dr / den, -di / den};
  }
  return r;
}

// component c >= k+1 of the Householder vector (v_{k+1} = 1)
__device__ inline double2 hh_v(int c, int k, double2 row_c, double2 sc) {
  return c == k + 1 ? double2{1.0, 0.0} : cmul(double2{row_c.x, -row_c.y}, sc);
}

// One exchange per column.  Every workgroup holds the current pivot row k
// (row k of the partly reduced matrix; column k below the diagonal is its
// conjugate) and derives the reflector H_k from it.  The row owners publish
// x = tau A v; the owner of row k+1 also publishes that row, from which every
// workgroup forms the next pivot row by the rank-2 update (and, in the same
// pass, the norm that the next reflector needs).  Published buffers alternate
// between two copies, tagged k + 1: a workgroup publishes column k + 1 only
// after it has read everything of column k, so no copy is overwritten while
// a reader still needs it.
template <int NMAX, int LDS, bool QLDS>
__global__ __launch_bounds__(TNT) void tridiag_kernel(TdBatch batch) {
  __shared__ double sred[TNT / 64];     // per-wave |row[k+2:]|^2 of the pivot row
  __shared__ double2 s_xv[TNT / 64];    // per-wave parts of x^H v
  __shared__ int s_fail;

  int sec = 0;
  while (sec + 1 < batch.nsec && batch.wg0[sec + 1] <= (int)blockIdx.x) ++sec;
  const TdArgs a = batch.sec[sec];
  // A rows [R][n] (then, QLDS, Q rows [R][n]) and the vectors v, w and the
  // pivot row: fixed arrays for n <= 512; for the larger matrices sized to
  // the launch (R n + 3 n complex), so that two workgroups share a CU up to
  // n ~ 730
  double2 *sM, *sv, *sw, *srow;
  if constexpr (QLDS) {
    __shared__ double2 fM[LDS];
    __shared__ double2 fv[NMAX], fw[NMAX], frow[NMAX];
    sM = fM;
    sv = fv;
    sw = fw;
    srow = frow;
  } else {
    extern __shared__ double2 td_dyn[];
    sM = td_dyn;
    sv = td_dyn + (size_t)a.R * a.n;
    sw = sv + a.n;
    srow = sw + a.n;
  }
  const int n = a.n, G = a.G, R = a.R, g = (int)blockIdx.x - batch.wg0[sec], tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  double2* sA = sM;
  // Q row j of this workgroup: in LDS, or row g + j G of the output
  auto qrow_at = [&](int j) -> double2* {
    return QLDS ? sM + (size_t)R * n + (size_t)j * n : a.Q + (size_t)(g + j * G) * n;
  };
  const int nrow = (n - g + G - 1) / G;   // rows r = g + j G < n
  // T threads per own row (a power of two, within one wave): thread tid works
  // on local row rj = tid / T, columns rt, rt + T, ...
  int T = 64;
  while (T > 1 && T * R > TNT) T >>= 1;
  const int rj = tid / T, rt = tid % T;

  // own rows, Q = I, pivot row 0 and its norm beyond column 1
  for (int j = 0; j < nrow; ++j) {
    const int r = g + j * G;
    for (int c = tid; c < n; c += TNT) {
      sA[j * n + c] = a.H[(size_t)r * n + c];
      qrow_at(j)[c] = double2{r == c ? 1.0 : 0.0, 0.0};
    }
  }
  {
    double ssq = 0.0;
    for (int c = tid; c < n; c += TNT) {
      const double2 h = a.H[c];
      srow[c] = h;
      if (c >= 2) ssq += h.x * h.x + h.y * h.y;
    }
    ssq = wave::sum(ssq);
    if (lane == 0) sred[wave] = ssq;
  }
  if (tid == 0) s_fail = 0;
  __syncthreads();

  bool alive = true;
  for (int k = 0; k + 1 < n; ++k) {
    const int par = k & 1;
    double xn2 = 0.0;
#pragma unroll
    for (int w = 0; w < TNT / 64; ++w) xn2 += sred[w];
    const Reflector hr = reflector(srow[k + 1], xn2);
    const double2 tau = hr.tau, sc = hr.sc;
    if (g == 0 && tid == 0) {
      a.D[k] = srow[k].x;
      a.E[k] = hr.beta;
    }

    // ---- one pass over the own rows (T threads per row): x = tau A v for
    // rows >= k+1 and tau (Q v) for the accumulation of Q.
    // v is formed on the fly (the threads of local row 0 also store it).
    // The owner of row k+1 publishes it (before this column's update).
    const unsigned tag = (unsigned)k + 1u;
    unsigned long long* xvp = a.xv + (size_t)par * 4 * n;
    unsigned long long* rowp = a.prow + (size_t)par * 4 * n;
    double2 tqs{0.0, 0.0};
    if (rj < nrow) {
      double2 sa{0.0, 0.0}, sq{0.0, 0.0};
      const double2* arow = sA + rj * n;
      const double2* qrow = qrow_at(rj);
      for (int c = k + 1 + rt; c < n; c += T) {
        const double2 v = hh_v(c, k, srow[c], sc), m = arow[c], q = qrow[c];
        if (rj == 0) sv[c] = v;
        sa.x += m.x * v.x - m.y * v.y;
        sa.y += m.x * v.y + m.y * v.x;
        sq.x += q.x * v.x - q.y * v.y;
        sq.y += q.x * v.y + q.y * v.x;
      }
      sa.x = wave::group_sum(sa.x, T);
      sa.y = wave::group_sum(sa.y, T);
      sq.x = wave::group_sum(sq.x, T);
      sq.y = wave::group_sum(sq.y, T);
      tqs = cmul(tau, sq);
      const int r = g + rj * G;
      if (rt == 0 && r >= k + 1) put_tagged(xvp + 4 * (size_t)r, cmul(tau, sa), tag);
    }
    if ((k + 1) % G == g) {
      const int j = (k + 1) / G;
      for (int c = k + 1 + tid; c < n; c += TNT) put_tagged(rowp + 4 * (size_t)c, sA[j * n + c], tag);
    }
    __syncthreads();

    // ---- while the others arrive: Q <- Q H_k = Q - tau (Q v) v^H on the own rows
    if (rj < nrow) {
      double2* qrow = qrow_at(rj);
      for (int c = k + 1 + rt; c < n; c += T) {
        const double2 d = cmulc(tqs, sv[c]);
        qrow[c].x -= d.x;
        qrow[c].y -= d.y;
      }
    }
    // ---- gather this column's x and pivot row as they arrive (every thread
    // its own entries)
    constexpr int NQ = (NMAX + TNT - 1) / TNT;
    double2 xq[NQ], rq[NQ];
    {
      bool gx[NQ], gr[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c = k + 1 + tid + q * TNT;
        gx[q] = gr[q] = c >= n;
        xq[q] = rq[q] = double2{0.0, 0.0};
      }
      unsigned polls = 0;
      while (true) {
        bool done = true;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int c = k + 1 + tid + q * TNT;
          if (!gx[q]) gx[q] = get_tagged(xvp + 4 * (size_t)c, tag, &xq[q]);
          if (!gr[q]) gr[q] = get_tagged(rowp + 4 * (size_t)c, tag, &rq[q]);
          done = done && gx[q] && gr[q];
        }
        if (done) break;
        ++polls;
        if (polls > SPIN_LIMIT ||
            ((polls & 63u) == 0 && __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
          __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_fail = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    {   // x^H v from the gathered x: own entries, the wave, then the waves in order
      double2 pv{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c = k + 1 + tid + q * TNT;
        if (c < n) {
          const double2 v = sv[c];
          pv.x += xq[q].x * v.x + xq[q].y * v.y;
          pv.y += xq[q].x * v.y - xq[q].y * v.x;
        }
      }
      pv = wave_sum(pv);
      if (lane == 0) s_xv[wave] = pv;
    }
    __syncthreads();
    if (s_fail) {
      alive = false;
      break;
    }

    // ---- w = x - (tau/2)(x^H v) v; next pivot row and its norm beyond
    // column k+2; A <- A - v w^H - w v^H on the own rows
    {
      double2 t = s_xv[0];
#pragma unroll
      for (int w = 1; w < TNT / 64; ++w) {
        t.x += s_xv[w].x;
        t.y += s_xv[w].y;
      }
      const double2 a2x = cmul(tau, t);
      const double2 a2{-0.5 * a2x.x, -0.5 * a2x.y};
#pragma unroll
      for (int q = 0; q < (NMAX + TNT - 1) / TNT; ++q) {
        const int c = k + 1 + tid + q * TNT;
        if (c < n) {
          const double2 tv = cmul(a2, sv[c]);
          sw[c] = double2{xq[q].x + tv.x, xq[q].y + tv.y};
        }
      }
      __syncthreads();
      const double2 v1 = sv[k + 1], w1 = sw[k + 1];
      double ssq = 0.0;
#pragma unroll
      for (int q = 0; q < (NMAX + TNT - 1) / TNT; ++q) {
        const int c = k + 1 + tid + q * TNT;
        if (c < n) {
          const double2 d1 = cmulc(v1, sw[c]), d2 = cmulc(w1, sv[c]);
          const double2 nr{rq[q].x - (d1.x + d2.x), rq[q].y - (d1.y + d2.y)};
          srow[c] = nr;
          if (c >= k + 3) ssq += nr.x * nr.x + nr.y * nr.y;
        }
      }
      ssq = wave::sum(ssq);
      if (lane == 0) sred[wave] = ssq;
    }
    if (rj < nrow && g + rj * G >= k + 2) {   // rows <= k+1 are finished
      const int r = g + rj * G;
      const double2 vr = sv[r], wr = sw[r];
      double2* arow = sA + rj * n;
      for (int c = k + 1 + rt; c < n; c += T) {
        const double2 d1 = cmulc(vr, sw[c]), d2 = cmulc(wr, sv[c]);
        arow[c].x -= d1.x + d2.x;
        arow[c].y -= d1.y + d2.y;
      }
    }
    __syncthreads();
  }

  if (alive) {
    if (g == 0 && tid == 0) a.D[n - 1] = srow[n - 1].x;
    if (QLDS)
      for (int j = 0; j < nrow; ++j) {
        const int r = g + j * G;
        for (int c = tid; c < n; c += TNT) a.Q[(size_t)r * n + c] = qrow_at(j)[c];
      }
  }
}

// rows[j][m] = Z[m][n-1-j] as complex, Z column-major real (eigenvector j'
// contiguous): the eigenvectors of the tridiagonal matrix in descending order
__global__ void zrows_from_real_kernel(double2* __restrict__ out, const double* __restrict__ Z, int n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  const int j = (int)(idx / n), m = (int)(idx % n);
  out[idx] = double2{Z[(size_t)(n - 1 - j) * n + m], 0.0};
}

// G <- G - frac * tr(G) I for a Hermitian n x n matrix (one workgroup)
// G = S - frac trace(S) I.  With G == S one workgroup shifts the diagonal;
// otherwise every workgroup finds the same trace (the same order) and copies
// its share of the entries, shifting those on the diagonal.
__global__ __launch_bounds__(TNT) void shift_by_trace_kernel(double2* G, const double2* S, int n, double frac) {
  __shared__ double red[TNT / 64];
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += TNT) t += S[(size_t)i * n + i].x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  double tr = 0.0;
  for (int w = 0; w < TNT / 64; ++w) tr += red[w];
  const double mu = frac * tr;
  if (G == S) {
    for (int i = threadIdx.x; i < n; i += TNT) G[(size_t)i * n + i].x -= mu;
    return;
  }
  const long long nn = (long long)n * n;
  for (long long e = (long long)blockIdx.x * TNT + threadIdx.x; e < nn; e += (long long)gridDim.x * TNT) {
    double2 v = S[e];
    if (e / n == e % n) v.x -= mu;
    G[e] = v;
  }
}

// the tagged exchange words of up to TD_RESET_MAX sectors (problem y of
// the launch: nw[y] words at w[y]) and the shared error flag
constexpr int TD_RESET_MAX = 64;
struct TdReset {
  int n;
  int* err;
  unsigned* w[TD_RESET_MAX];
  int nw[TD_RESET_MAX];
};
__global__ void td_reset_kernel(const TdReset r) {
  const int y = blockIdx.y;
  if (y >= r.n) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < r.nw[y]; i += gridDim.x * blockDim.x) r.w[y][i] = 0u;
  if (y == 0 && blockIdx.x == 0 && threadIdx.x == 0 && r.err) *r.err = 0;
}

// ------------------------------------------------ charge blocks side by side
// Block y of the launch (kern::EigBlock) holds indices idx[off .. off + m) of
// the n x n matrix; every kernel walks its m x m entries with a grid-stride
// loop over blockIdx.x.
constexpr int EB_MAX = 64;
struct EigBlockBatch {
  int n;
  kern::EigBlock b[EB_MAX];
};
static_assert(sizeof(EigBlockBatch) <= 4096 && sizeof(TdReset) <= 4096, "kernel arguments too large");

// X = (H_b + H_b^H) / 2 of the gathered block (the diagonal's imaginary part
// dropped), as a gather followed by zhermitize would give it
__global__ void eb_gather_kernel(const EigBlockBatch bt, const double2* __restrict__ H, long long n,
                                 const int* __restrict__ idx) {
  const int y = blockIdx.y;
  if (y >= bt.n) return;
  const kern::EigBlock e = bt.b[y];
  const long long mm = (long long)e.m * e.m;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < mm; t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t / e.m), j = (int)(t % e.m);
    const long long ri = idx[e.off + i], rj = idx[e.off + j];
    const double2 a = H[ri * n + rj];
    if (i == j) {
      e.X[t] = make_double2(a.x, 0.0);
    } else {
      const double2 b = H[rj * n + ri];
      e.X[t] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    }
  }
}

// X[j][k] = Z[k][m-1-j] (real eigenvectors, column-major ascending -> rows, descending)
__global__ void eb_rows_kernel(const EigBlockBatch bt) {
  const int y = blockIdx.y;
  if (y >= bt.n) return;
  const kern::EigBlock e = bt.b[y];
  const long long mm = (long long)e.m * e.m;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < mm; t += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(t / e.m), k = (int)(t % e.m);
    e.X[t] = double2{e.Z[(size_t)(e.m - 1 - j) * e.m + k], 0.0};
  }
}

// sums[y] = sum |R_y|^2 (one workgroup per block; the check of the back
// transformation: m for orthonormal rows)
__global__ __launch_bounds__(TNT) void eb_norms_kernel(const EigBlockBatch bt, double2* __restrict__ sums) {
  __shared__ double red[TNT / 64];
  const int y = blockIdx.y;
  if (y >= bt.n) return;
  const kern::EigBlock e = bt.b[y];
  const long long mm = (long long)e.m * e.m;
  double acc = 0.0;
  for (long long t = threadIdx.x; t < mm; t += TNT) acc += e.R[t].x * e.R[t].x + e.R[t].y * e.R[t].y;
  acc = wave::sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < TNT / 64; ++w) tot += red[w];
    sums[y] = make_double2(tot, 0.0);
  }
}

// rows[off + i][idx[off + j]] = R[i][j]
__global__ void eb_scatter_kernel(const EigBlockBatch bt, double2* __restrict__ rows, long long n,
                                  const int* __restrict__ idx) {
  const int y = blockIdx.y;
  if (y >= bt.n) return;
  const kern::EigBlock e = bt.b[y];
  const long long mm = (long long)e.m * e.m;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < mm; t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t / e.m), j = (int)(t % e.m);
    rows[(long long)(e.off + i) * n + idx[e.off + j]] = e.R[t];
  }
}

// grid x for an m x m walk (capped: the loops stride)
unsigned eb_grid_x(const kern::EigBlock* blk, int nb) {
  long long mx = 1;
  for (int i = 0; i < nb; ++i) mx = std::max(mx, (long long)blk[i].m * blk[i].m);
  return (unsigned)std::min<long long>(1024, (mx + 255) / 256);
}

}  // namespace

namespace kern {

int tridiag_groups(int n) {
  if (n > TD_NMAX && n <= TD_NMAX_BIG) {
    const int G = std::min(TD_G_BIG, (n + 3) / 4);
    const int R = (n + G - 1) / G;
    return R * n <= TD_LDS_BIG ? G : 0;
  }
  if (n < 1 || n > TD_NMAX) return 0;
  // The per-column work of a workgroup grows with its share of the rows and
  // the exchange with the number of workgroups: four rows per workgroup (one
  // wave per row) is fastest at every n measured, 8 to 512 (eight rows are
  // 8-15% slower from n = 64 on, two no faster, one workgroup for n <= 32 up
  // to 25% slower).  At most 128 workgroups, and 2 R n complex slots of LDS
  // for the A and Q rows.
  const int G = std::min(128, (n + 3) / 4);
  const int R = (n + G - 1) / G;
  return (2 * R * n <= TD_LDS && R <= TD_ROWS) ? G : 0;
}

size_t tridiag_scratch_bytes(int n) {
  const int G = tridiag_groups(n);
  return G == 0 ? 0 : sizeof(unsigned long long) * 4 * 4 * (size_t)n + 256;
}

hipError_t tridiag(hipStream_t s, const void* H, int n, void* Q, double* D, double* E, void* scratch, int* err) {
  if (tridiag_groups(n) == 0) return hipErrorInvalidValue;
  const TdSector one{H, Q, D, E, scratch, n};
  return tridiag_batched(s, &one, 1, err);
}

// Workgroups of the sectors of one launch (every workgroup holds one CU's
// worth of LDS, so at most TD_WG_LAUNCH): each sector gets at least the
// workgroups its LDS share needs, the rest go where the work per workgroup
// (~ n^3 / G) is largest, up to four rows per workgroup.
namespace {
constexpr int TD_WG_LAUNCH = 256;
int td_rmax(int n) { return n > TD_NMAX ? 4 : std::min(TD_ROWS, TD_LDS / (2 * n)); }
int td_gmin(int n) { return (n + td_rmax(n) - 1) / td_rmax(n); }
int td_gpref(int n) { return std::min(n > TD_NMAX ? TD_G_BIG : 128, (n + 3) / 4); }
// the larger variant: four rows per workgroup, LDS of R n + 3 n complex; as
// many workgroups per launch as fit the CUs' LDS (160 KiB each, at most 8
// workgroups of 256 threads)
size_t td_big_lds(int n) { return sizeof(double2) * (size_t)(4 * n + 3 * n); }
int td_big_cap(size_t lds) {
  const size_t per_cu = std::min<size_t>(8, (160 * 1024 - 256) / lds);
  return (int)(256 * std::max<size_t>(per_cu, 1));
}
}  // namespace

hipError_t tridiag_batched(hipStream_t s, const TdSector* sec, int nsec, int* err) {
  if (nsec < 1 || !err) return hipErrorInvalidValue;
  for (int i = 0; i < nsec; ++i)
    if (sec[i].n < 2 || sec[i].n > TD_NMAX_BIG || !sec[i].scratch) return hipErrorInvalidValue;
  // the tagged words of every sector, and the error flag once
  for (int i0 = 0; i0 < nsec; i0 += TD_RESET_MAX) {
    TdReset r{};
    r.err = i0 == 0 ? err : nullptr;
    int mx = 1;
    for (int i = i0; i < std::min(nsec, i0 + TD_RESET_MAX); ++i) {
      r.w[r.n] = static_cast<unsigned*>(sec[i].scratch);
      r.nw[r.n] = 2 * 4 * 4 * sec[i].n;   // 32-bit halves of the tagged words
      mx = std::max(mx, r.nw[r.n]);
      ++r.n;
    }
    hipLaunchKernelGGL(td_reset_kernel, dim3((unsigned)std::min(64, (mx + 255) / 256), r.n), dim3(256), 0, s, r);
  }
  // two variants (Q rows in LDS up to n = 512, in the output above); in
  // each, sectors in decreasing size packed into launches
  for (int big = 0; big < 2; ++big) {
    std::vector<int> ids;
    for (int i = 0; i < nsec; ++i)
      if ((sec[i].n > TD_NMAX) == (big == 1)) ids.push_back(i);
    std::stable_sort(ids.begin(), ids.end(), [&](int x, int y) { return sec[x].n > sec[y].n; });
    for (size_t k = 0; k < ids.size();) {
      std::vector<int> grp, G;
      int tot = 0;
      // the first (largest) sector sets the LDS of the launch
      const size_t lds = big ? td_big_lds(sec[ids[k]].n) : 0;
      const int cap = big ? td_big_cap(lds) : TD_WG_LAUNCH;
      while (k < ids.size() && (int)grp.size() < TD_MAXSEC &&
             (grp.empty() || tot + td_gmin(sec[ids[k]].n) <= cap)) {
        grp.push_back(ids[k]);
        G.push_back(td_gmin(sec[ids[k]].n));
        tot += G.back();
        ++k;
      }
      for (int spare = (big ? 0 : TD_WG_LAUNCH - tot); spare > 0; --spare) {
        int best = -1;
        double wbest = 0.0;
        for (size_t j = 0; j < grp.size(); ++j) {
          const double nn = sec[grp[j]].n, w = nn * nn * nn / G[j];
          if (G[j] < td_gpref(sec[grp[j]].n) && w > wbest) {
            wbest = w;
            best = (int)j;
          }
        }
        if (best < 0) break;
        ++G[best];
      }
      TdBatch b{};
      int wg = 0;
      for (size_t j = 0; j < grp.size(); ++j) {
        const TdSector& x = sec[grp[j]];
        TdArgs& a = b.sec[j];
        a.H = static_cast<const double2*>(x.H);
        a.Q = static_cast<double2*>(x.Q);
        a.D = x.D;
        a.E = x.E;
        a.xv = static_cast<unsigned long long*>(x.scratch);   // two buffers of n complex each
        a.prow = a.xv + 8 * (size_t)x.n;
        a.err = err;
        a.n = x.n;
        a.G = G[j];
        a.R = (x.n + G[j] - 1) / G[j];
        b.wg0[j] = wg;
        wg += G[j];
      }
      b.wg0[grp.size()] = wg;
      b.nsec = (int)grp.size();
      void* args[] = {&b};
      const void* kfn = big ? reinterpret_cast<const void*>(tridiag_kernel<TD_NMAX_BIG, TD_LDS_BIG, false>)
                            : reinterpret_cast<const void*>(tridiag_kernel<TD_NMAX, TD_LDS, true>);
      const hipError_t e = hipLaunchCooperativeKernel(kfn, dim3(wg), dim3(TNT), args, (unsigned)lds, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

void shift_by_trace(hipStream_t s, void* G, int n, double frac, const void* S) {
  if (n <= 0) return;
  const double2* src = S ? static_cast<const double2*>(S) : static_cast<const double2*>(G);
  const long long nn = (long long)n * n;
  const unsigned blocks = src == G ? 1u : (unsigned)std::min<long long>(256, (nn + TNT - 1) / TNT);
  hipLaunchKernelGGL(shift_by_trace_kernel, dim3(blocks), dim3(TNT), 0, s, static_cast<double2*>(G), src, n, frac);
}

void eig_blocks_gather(hipStream_t s, const EigBlock* blk, int nb, const void* H, long long n, const int* idx) {
  for (int g = 0; g < nb; g += EB_MAX) {
    EigBlockBatch bt{};
    bt.n = std::min(EB_MAX, nb - g);
    std::copy(blk + g, blk + g + bt.n, bt.b);
    hipLaunchKernelGGL(eb_gather_kernel, dim3(eb_grid_x(bt.b, bt.n), bt.n), dim3(256), 0, s, bt,
                       static_cast<const double2*>(H), n, idx);
  }
}

void eig_blocks_rows(hipStream_t s, const EigBlock* blk, int nb) {
  for (int g = 0; g < nb; g += EB_MAX) {
    EigBlockBatch bt{};
    bt.n = std::min(EB_MAX, nb - g);
    std::copy(blk + g, blk + g + bt.n, bt.b);
    hipLaunchKernelGGL(eb_rows_kernel, dim3(eb_grid_x(bt.b, bt.n), bt.n), dim3(256), 0, s, bt);
  }
}

void eig_blocks_norms(hipStream_t s, const EigBlock* blk, int nb, void* sums) {
  for (int g = 0; g < nb; g += EB_MAX) {
    EigBlockBatch bt{};
    bt.n = std::min(EB_MAX, nb - g);
    std::copy(blk + g, blk + g + bt.n, bt.b);
    hipLaunchKernelGGL(eb_norms_kernel, dim3(1, bt.n), dim3(TNT), 0, s, bt, static_cast<double2*>(sums) + g);
  }
}

void eig_blocks_scatter(hipStream_t s, const EigBlock* blk, int nb, void* rows, long long n, const int* idx) {
  for (int g = 0; g < nb; g += EB_MAX) {
    EigBlockBatch bt{};
    bt.n = std::min(EB_MAX, nb - g);
    std::copy(blk + g, blk + g + bt.n, bt.b);
    hipLaunchKernelGGL(eb_scatter_kernel, dim3(eb_grid_x(bt.b, bt.n), bt.n), dim3(256), 0, s, bt,
                       static_cast<double2*>(rows), n, idx);
  }
}

void zrows_from_real_desc(hipStream_t s, void* out, const double* Z, int n) {
  const long long nn = (long long)n * n;
  hipLaunchKernelGGL(zrows_from_real_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s,
                     static_cast<double2*>(out), Z, n);
}

}  // namespace kern
