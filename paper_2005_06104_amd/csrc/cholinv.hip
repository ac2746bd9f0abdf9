// Cholesky factorisation G = L L^H of a Hermitian positive definite n x n
// matrix (n <= 512, row-major complex128) together with L^-1, in one
// cooperative launch with one workgroup per 16 x 16 block (i, k), k <= i, of
// the lower triangle (tiled right-looking order, each update applied as soon
// as its operands exist):
//     L_ik = (G_ik - sum_{j<k} L_ij L_kj^H) (L_kk^-1)^H           k < i,
//     L_ii = chol(G_ii - sum_{j<i} L_ij L_ij^H),  with L_ii^-1,
//     Linv_ik = -L_ii^-1 sum_{j=k}^{i-1} L_ij Linv_jk              k < i.
// A block is published with a flag once written; a workgroup waits only for
// blocks of lower column index (or, for L^-1, of lower row index in its own
// column) and for diagonal blocks, so the waits form chains that end.  Only
// the diagonal chain (one factorisation and inversion of a 16 x 16 block and
// two block products per block row) is sequential: small blocks keep its
// column steps few and short.  Every wait is bounded;
// one that runs out makes the call report failure.  The factorisation
// reports failure when a pivot is not positive and finite.
// Block-diagonal matrices (the Gram matrices of charged tensors, whose
// charge sectors are contiguous) are factorised sector by sector in the same
// launch: each sector has its own workgroups and flags, and the blocks
// between sectors are never read.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace {

constexpr int CB = 16;            // block size
constexpr int CNT = 256;          // threads per workgroup
constexpr int CMAXB = 32;         // block rows at most
constexpr int CENT = CB * CB / CNT;   // tile entries per thread
constexpr int CPR = CNT / CB;         // threads per tile row
constexpr int NPART = 64 / CB;        // lanes per row in the one-wave steps
static_assert(CENT >= 1 && CB * CB == CENT * CNT && NPART >= 1, "tile mapping");
constexpr int CFLAG = 16;         // one 64-byte line per flag
constexpr unsigned CSPIN = 1u << 22;
constexpr int CMAXSEC = 64;       // sectors per launch
constexpr int CMAXWG = 1024;      // workgroups per launch (all co-resident)
constexpr size_t CSEC_FLAGS = 2 * CMAXB * CMAXB * CFLAG;   // flag words per sector

struct CholArgs {
  const double2* G;   // ld x ld, Hermitian (the lower blocks of each sector are read)
  double2* L;         // out: the lower blocks of L in each sector (may be G)
  double2* Li;        // out: L^-1 in each sector (zero above the diagonal)
  unsigned* flags;    // CSEC_FLAGS per sector, zero at launch
  int* info;          // 0 at launch; 1 not positive definite, 2 a wait ran out
  int ld, nsec;
  int off[CMAXSEC], size[CMAXSEC], wg0[CMAXSEC + 1];   // sector s: rows off..off+size, workgroups wg0[s]..
};

// one sector as the workgroup sees it
struct Sec {
  const double2* G;
  double2* L;
  double2* Li;
  unsigned* fl;       // block (i, k) of L published (k = i: with L_ii^-1)
  unsigned* fi;       // block (i, k) of L^-1 published (i > k)
  int* info;
  int n, ld;
};

__device__ inline double2 cm(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline double2 cmc(double2 a, double2 b) {   // a * conj(b)
  return double2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

__device__ inline int bsize(const Sec& a, int i) { return min(CB, a.n - i * CB); }

__device__ inline unsigned* flag_at(unsigned* f, int r, int c) { return f + (r * CMAXB + c) * CFLAG; }

// wait until the flags f1 and f2 are set; false when a wait ran out or
// another workgroup gave up
__device__ bool wait_flags(const Sec& a, const unsigned* f1, const unsigned* f2, int* s_ok) {
  if (threadIdx.x == 0) {
    unsigned polls = 0;
    int ok = 1;
    while (__hip_atomic_load(f1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u ||
           __hip_atomic_load(f2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      if (__hip_atomic_load(a.info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 2 || ++polls > CSPIN) {
        __hip_atomic_store(a.info, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// set flag f once the workgroup's stores before the call are done
__device__ void publish(unsigned* f) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// tile[r][c] = M[(r0 + r) * n + c0 + c] for r < rows, c < cols; zero elsewhere
__device__ void load_tile(double2 (*t)[CB + 1], const double2* M, int n, int r0, int rows, int c0, int cols) {
  for (int e = threadIdx.x; e < CB * CB; e += CNT) {
    const int r = e / CB, c = e % CB;
    t[r][c] = (r < rows && c < cols) ? M[(size_t)(r0 + r) * n + c0 + c] : double2{0.0, 0.0};
  }
}

__device__ void store_tile(const double2 (*t)[CB + 1], double2* M, int n, int r0, int rows, int c0, int cols) {
  for (int e = threadIdx.x; e < CB * CB; e += CNT) {
    const int r = e / CB, c = e % CB;
    if (r < rows && c < cols) M[(size_t)(r0 + r) * n + c0 + c] = t[r][c];
  }
}

// acc[q] (the thread's entries of a tile: row tid / CPR, columns
// (tid % CPR) + CPR q) += sign * (X Y^H) or sign * (X Y)
template <bool HERM>
__device__ void tile_mma(double2 acc[CENT], const double2 (*X)[CB + 1], const double2 (*Y)[CB + 1], double sign) {
  const int r = threadIdx.x / CPR, c0 = threadIdx.x % CPR;
#pragma unroll 4
  for (int k = 0; k < CB; ++k) {
    const double2 x = X[r][k];
#pragma unroll
    for (int q = 0; q < CENT; ++q) {
      const int c = c0 + CPR * q;
      const double2 p = HERM ? cmc(x, Y[c][k]) : cm(x, Y[k][c]);
      acc[q].x += sign * p.x;
      acc[q].y += sign * p.y;
    }
  }
}

__device__ void acc_to_tile(const double2 acc[CENT], double2 (*t)[CB + 1]) {
  const int r = threadIdx.x / CPR, c0 = threadIdx.x % CPR;
#pragma unroll
  for (int q = 0; q < CENT; ++q) t[r][c0 + CPR * q] = acc[q];
}

__device__ void tile_to_acc(const double2 (*t)[CB + 1], double2 acc[CENT]) {
  const int r = threadIdx.x / CPR, c0 = threadIdx.x % CPR;
#pragma unroll
  for (int q = 0; q < CENT; ++q) acc[q] = t[r][c0 + CPR * q];
}

// Wave 0 factorises the mi x mi block in tS (the lower part; the strict upper
// part holds the matrix) in place and forms its inverse in tY; *s_fail
// becomes 1 when a pivot is not positive and finite.  The lanes of one wave
// see each other's LDS stores in program order, so the steps need no
// workgroup barrier.
__device__ void diag_chol_inv(double2 (*tS)[CB + 1], double2 (*tY)[CB + 1], int mi, int* s_fail) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int bad = 0;
    // left-looking: column c of L from the dot products of the rows r >= c
    // with row c over the finished columns (row r on the NPART lanes
    // r + CB p, each adding every NPART-th term)
    const int rr = lane % CB, part = lane / CB;
    for (int c = 0; c < mi; ++c) {
      double2 t{0.0, 0.0};
      if (rr >= c && rr < mi)
        for (int k = part; k < c; k += NPART) {
          const double2 p = cmc(tS[rr][k], tS[c][k]);
          t.x += p.x;
          t.y += p.y;
        }
#pragma unroll
      for (int o = CB; o < 64; o <<= 1) {
        t.x += __shfl_xor(t.x, o);
        t.y += __shfl_xor(t.y, o);
      }
      const double d = tS[c][c].x - __shfl(t.x, c);
      const bool good = d > 0.0 && isfinite(d);
      bad |= good ? 0 : 1;
      const double l = good ? sqrt(d) : 1.0, il = 1.0 / l;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (part == 0 && rr > c && rr < mi) {
        const double2 v = tS[rr][c];
        tS[rr][c] = double2{(v.x - t.x) * il, (v.y - t.y) * il};
      }
      if (lane == c) tS[c][c] = double2{l, 0.0};
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // zero above the diagonal and outside the block
    for (int e = lane; e < CB * CB; e += 64) {
      const int r = e / CB, c = e % CB;
      if (c > r || r >= mi || c >= mi) tS[r][c] = double2{0.0, 0.0};
      tY[r][c] = double2{0.0, 0.0};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // L^-1 by forward substitution, column j on the NPART lanes j + CB p
    // (each adds every NPART-th term; shuffles join them)
    {
      const int j = lane % CB, part = lane / CB;
      const bool act = j < mi;
      double2 xj = double2{0.0, 0.0};
      if (act && part == 0) {
        xj = double2{1.0 / tS[j][j].x, 0.0};
        tY[j][j] = xj;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int r = 1; r < mi; ++r) {
        // x_r (column j, r > j) = -(sum_{s=j}^{r-1} L[r][s] x_s) / L[r][r]
        double2 t{0.0, 0.0};
        if (act && r > j)
          for (int q = j + part; q < r; q += NPART) {
            const double2 p = cm(tS[r][q], tY[q][j]);
            t.x += p.x;
            t.y += p.y;
          }
#pragma unroll
        for (int o = CB; o < 64; o <<= 1) {
          t.x += __shfl_xor(t.x, o);
          t.y += __shfl_xor(t.y, o);
        }
        if (act && r > j && part == 0) {
          const double ir = 1.0 / tS[r][r].x;
          tY[r][j] = double2{-t.x * ir, -t.y * ir};
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    if (lane == 0) *s_fail = bad;
  }
}

__global__ __launch_bounds__(CNT) void cholinv_kernel(CholArgs args) {
  __shared__ double2 tS[CB][CB + 1], tX[CB][CB + 1], tY[CB][CB + 1];
  __shared__ int s_ok, s_fail;
  int sec = 0;
  while (sec + 1 < args.nsec && args.wg0[sec + 1] <= (int)blockIdx.x) ++sec;
  const int wg = (int)blockIdx.x - args.wg0[sec];
  Sec a;
  {
    const size_t o = (size_t)args.off[sec] * args.ld + args.off[sec];
    a.G = args.G + o;
    a.L = args.L + o;
    a.Li = args.Li + o;
    a.fl = args.flags + sec * CSEC_FLAGS;
    a.fi = a.fl + CMAXB * CMAXB * CFLAG;
    a.info = args.info;
    a.n = args.size[sec];
    a.ld = args.ld;
  }
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= wg) ++i;
  const int k = wg - i * (i + 1) / 2;
  const int n = a.ld, mi = bsize(a, i), mk = bsize(a, k), ri = i * CB, rk = k * CB;
  double2 acc[CENT];

  // ---- S = G_ik - sum_{j<k} L_ij L_kj^H (blocks j < k are full)
  load_tile(tS, a.G, n, ri, mi, rk, mk);
  __syncthreads();
  tile_to_acc(tS, acc);
  for (int j = 0; j < k; ++j) {
    if (!wait_flags(a, flag_at(a.fl, i, j), flag_at(a.fl, k, j), &s_ok)) return;
    load_tile(tX, a.L, n, ri, mi, j * CB, CB);                     // L_ij
    if (i != k) load_tile(tY, a.L, n, rk, mk, j * CB, CB);         // L_kj
    __syncthreads();
    tile_mma<true>(acc, tX, i == k ? tX : tY, -1.0);
    __syncthreads();
  }

  if (i == k) {
    // ---- diagonal block: L_ii and L_ii^-1
    acc_to_tile(acc, tS);
    if (threadIdx.x == 0) s_fail = 0;
    __syncthreads();
    diag_chol_inv(tS, tY, mi, &s_fail);
    __syncthreads();
    store_tile(tS, a.L, n, ri, mi, ri, mi);
    store_tile(tY, a.Li, n, ri, mi, ri, mi);
    if (s_fail && threadIdx.x == 0) __hip_atomic_store(a.info, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    publish(flag_at(a.fl, i, i));
    return;
  }

  // ---- L_ik = S (L_kk^-1)^H, kept in tX
  if (!wait_flags(a, flag_at(a.fl, k, k), flag_at(a.fl, k, k), &s_ok)) return;
  acc_to_tile(acc, tS);
  load_tile(tY, a.Li, n, rk, mk, rk, mk);                            // L_kk^-1
  __syncthreads();
  for (int q = 0; q < CENT; ++q) acc[q] = double2{0.0, 0.0};
  tile_mma<true>(acc, tS, tY, 1.0);
  acc_to_tile(acc, tX);
  __syncthreads();
  store_tile(tX, a.L, n, ri, mi, rk, mk);
  publish(flag_at(a.fl, i, k));
  for (int e = threadIdx.x; e < CB * CB; e += CNT) {                   // block (k, i) of L^-1
    const int y = e / CB, x = e % CB;
    if (y < mk && x < mi) a.Li[(size_t)(rk + y) * n + ri + x] = double2{0.0, 0.0};
  }

  // ---- Linv_ik = -L_ii^-1 sum_{j=k}^{i-1} L_ij Linv_jk (blocks j < i are full)
  for (int q = 0; q < CENT; ++q) acc[q] = double2{0.0, 0.0};
  tile_mma<false>(acc, tX, tY, 1.0);                                 // j = k: L_ik L_kk^-1
  __syncthreads();
  for (int j = k + 1; j < i; ++j) {
    if (!wait_flags(a, flag_at(a.fl, i, j), flag_at(a.fi, j, k), &s_ok)) return;
    load_tile(tX, a.L, n, ri, mi, j * CB, CB);                       // L_ij
    load_tile(tY, a.Li, n, j * CB, CB, rk, mk);                      // Linv_jk
    __syncthreads();
    tile_mma<false>(acc, tX, tY, 1.0);
    __syncthreads();
  }
  if (!wait_flags(a, flag_at(a.fl, i, i), flag_at(a.fl, i, i), &s_ok)) return;
  acc_to_tile(acc, tS);
  load_tile(tX, a.Li, n, ri, mi, ri, mi);                            // L_ii^-1
  __syncthreads();
  for (int q = 0; q < CENT; ++q) acc[q] = double2{0.0, 0.0};
  tile_mma<false>(acc, tX, tS, -1.0);
  acc_to_tile(acc, tY);
  __syncthreads();
  store_tile(tY, a.Li, n, ri, mi, rk, mk);
  publish(flag_at(a.fi, i, k));
}

__global__ void cholinv_reset_kernel(unsigned* flags, int nf, int* info) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nf) flags[t] = 0u;
  if (t == 0 && info) *info = 0;
}

}  // namespace

namespace kern {

int cholinv_max_n() { return CB * CMAXB; }

size_t cholinv_scratch_bytes() { return sizeof(unsigned) * CSEC_FLAGS + 256; }

size_t cholinv_blocks_scratch_bytes() { return sizeof(unsigned) * CSEC_FLAGS * CMAXSEC + 256; }

hipError_t cholinv(hipStream_t s, const void* G, int n, void* L, void* Linv, int* info, void* scratch) {
  const int off = 0;
  return cholinv_blocks(s, G, n, &off, &n, 1, L, Linv, info, scratch, false);
}

hipError_t cholinv_blocks(hipStream_t s, const void* G, int ld, const int* off, const int* size, int nsec, void* L,
                          void* Linv, int* info, void* scratch, bool keep_info) {
  if (ld < 1 || nsec < 1 || !scratch || !info) return hipErrorInvalidValue;
  for (int q = 0; q < nsec; ++q)
    if (size[q] < 1 || size[q] > CB * CMAXB || off[q] < 0 || off[q] + size[q] > ld) return hipErrorInvalidValue;
  // sectors go to launches of at most CMAXSEC sectors and CMAXWG workgroups
  bool first = true;
  for (int q0 = 0; q0 < nsec;) {
    CholArgs a{};
    a.G = static_cast<const double2*>(G);
    a.L = static_cast<double2*>(L);
    a.Li = static_cast<double2*>(Linv);
    a.flags = static_cast<unsigned*>(scratch);
    a.info = info;
    a.ld = ld;
    int wg = 0, q = q0;
    while (q < nsec && a.nsec < CMAXSEC) {
      const int nb = (size[q] + CB - 1) / CB, w = nb * (nb + 1) / 2;
      if (a.nsec > 0 && wg + w > CMAXWG) break;
      a.off[a.nsec] = off[q];
      a.size[a.nsec] = size[q];
      a.wg0[a.nsec] = wg;
      wg += w;
      ++a.nsec;
      ++q;
    }
    a.wg0[a.nsec] = wg;
    // flags of the sectors used; info once per call (a failure in an earlier
    // launch stays reported) unless the caller cleared it
    const int nf = (int)(CSEC_FLAGS * a.nsec);
    hipLaunchKernelGGL(cholinv_reset_kernel, dim3((nf + 255) / 256), dim3(256), 0, s, a.flags, nf,
                       first && !keep_info ? a.info : nullptr);
    void* args[] = {&a};
    const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(cholinv_kernel), dim3(wg),
                                                    dim3(CNT), args, 0, s);
    if (e != hipSuccess) return e;
    first = false;
    q0 = q;
  }
  return hipSuccess;
}

}  // namespace kern
