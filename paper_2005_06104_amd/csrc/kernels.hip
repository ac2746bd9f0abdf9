// Device kernels of the GSE-TDVP1 hot path (gfx950 / CDNA4).
//
// * zgemm/cgemm: complex GEMM split into real MFMA products.  A complex
//   product (Ar + i Ai)(Br + i Bi) is three real MFMA accumulations,
//   Ar Br, Ai Bi and (Ar + Ai)(Br + Bi), combined into Ar Br - Ai Bi and
//   Ar Bi + Ai Br at the store; operand tiles are de-interleaved into real
//   and imaginary planes in LDS.
//   FP64 uses v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32 (same lane
//   layout).  These carry every contraction of the method: effective
//   Hamiltonians, environments, MPO application, basis extension.
// * wapply: contraction with the sparse MPO tensor over (MPO index, physical
//   index), staged through LDS; memory bound.
// * complex128 vector helpers for the Lanczos recurrence (FP64 always).
#include <hip/hip_runtime.h>

#include "common.h"
#include "wave.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct VT;
template <> struct VT<double> { using c2 = double2; using acc = d4; };
template <> struct VT<float> { using c2 = float2; using acc = f4; };

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- GEMM
// Block tile BM x BN complex outputs, BK complex per stage.  FP64: 1024
// threads = 16 waves in a 4 x 4 grid, one 16x16 MFMA tile each (four waves
// per SIMD keep the long FP64 MFMA pipeline fed while others wait on LDS or
// the stage barrier); FP32: 256 threads = 4 waves in a 2 x 2 grid, each
// 32 x 32 outputs = 2 x 2 MFMA tiles, for the real and for the imaginary part.
constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
constexpr int PAD = 1;
template <typename T> struct WaveGrid { static constexpr int WM = 2, WN = 2; };
template <> struct WaveGrid<double> { static constexpr int WM = 4, WN = 4; };
template <typename T> constexpr int gemm_threads() { return WaveGrid<T>::WM * WaveGrid<T>::WN * 64; }

// TAG only separates instantiations (the one-site effective Hamiltonian uses
// its own so that profilers and timers see it apart from the other GEMMs).
// Split-K: blockIdx.z = batch * S + split; split s covers k in
// [s*Kc, min(K, (s+1)*Kc)) and writes its partial product at C + s*sps.
// Block-sparse products (operands with U(1) charges): a linear grid over
// the work items kit (kern::KMap): item {tile, part, a, b} is output tile
// `tile` (batch entry outer) over the K intervals kiv[a .. b) as [x, y)
// pairs, its partial product at C + part * sps.  kit null: the dense tile
// grid over the whole K range (or one split-K part).  A tile with no
// interval writes alpha * 0 + beta * C.
struct KIter {
  const int2* iv;
  int n;
  int2 one;
  __device__ int2 at(int v) const { return iv ? iv[v] : one; }
};

// the output tile, batch entry, split part and K range of this workgroup,
// and the rows r0 .. r1, columns c0 .. c1 of the tile it computes
struct TileJob {
  int m0, n0, split;
  int r0, r1, c0, c1;
  long long bz;
  KIter kr;
};

__device__ inline TileJob tile_job(int M, int N, int K, int S, int Kc, const int4* __restrict__ kit,
                                   const int2* __restrict__ kiv) {
  TileJob j;
  const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if (kit) {
    // items in decreasing K length: dispatch order (and the XCD round robin
    // of consecutive workgroups) spreads the long ones
    const int4 it = kit[2 * (size_t)lin], rg = kit[2 * (size_t)lin + 1];
    const int gxt = (N + BN - 1) / BN, tpb = gxt * ((M + BM - 1) / BM);
    j.bz = it.x / tpb;
    const int trem = it.x % tpb;
    j.m0 = (trem / gxt) * BM;
    j.n0 = (trem % gxt) * BN;
    j.split = it.y;
    j.r0 = rg.x;
    j.r1 = rg.y;
    j.c0 = rg.z;
    j.c1 = rg.w;
    j.kr.iv = kiv + it.z;
    j.kr.n = it.w - it.z;
    j.kr.one = make_int2(0, 0);
    return j;
  }
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
  // linear id g runs on XCD g % 8.  Give each XCD a contiguous band of tiles
  // (z-slice, then tile row, then tile column) so that the operand panels a
  // band needs stay in that XCD's L2.
  const unsigned tot = gx * gy * gz;
  const unsigned t = (tot % 8u == 0u) ? (lin % 8u) * (tot / 8u) + lin / 8u : lin;
  const unsigned tz = t / (gx * gy), trem = t % (gx * gy);
  j.m0 = (int)(trem / gx) * BM;
  j.n0 = (int)(trem % gx) * BN;
  j.bz = tz / S;
  j.split = tz % S;
  j.r0 = 0;
  j.r1 = BM;
  j.c0 = 0;
  j.c1 = BN;
  const int kb = j.split * Kc, ke = min(K, kb + Kc);
  j.kr.iv = nullptr;
  j.kr.n = kb < ke ? 1 : 0;
  j.kr.one = make_int2(kb, ke);
  return j;
}

template <typename T, bool TA, bool CA, bool TB, bool CB, int TAG>
__global__ __launch_bounds__(gemm_threads<T>()) void gemm_kernel(int M, int N, int K, T ar, T ai, const T* __restrict__ A,
                                                   long long lda, long long sa, const T* __restrict__ B,
                                                   long long ldb, long long sb, T br, T bi,
                                                   T* __restrict__ C, long long ldc, long long sc, int S, int Kc,
                                                   long long sps, const int4* __restrict__ kit,
                                                   const int2* __restrict__ kiv) {
  using c2 = typename VT<T>::c2;
  using acc_t = typename VT<T>::acc;
  __shared__ T As_r[2][BK][BM + PAD], As_i[2][BK][BM + PAD];
  __shared__ T Bs_r[2][BK][BN + PAD], Bs_i[2][BK][BN + PAD];

  constexpr int WM = WaveGrid<T>::WM, WN = WaveGrid<T>::WN, NTH = WM * WN * 64;
  constexpr int SI = BM / WM / 16, SJ = BN / WN / 16;   // MFMA tiles per wave
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const TileJob job = tile_job(M, N, K, S, Kc, kit, kiv);
  const int m0 = job.m0, n0 = job.n0, split = job.split;
  const long long bz = job.bz;
  const c2* Ab = reinterpret_cast<const c2*>(A) + bz * sa;
  const c2* Bb = reinterpret_cast<const c2*>(B) + bz * sb;
  c2* Cb = reinterpret_cast<c2*>(C) + bz * sc + split * sps;

  constexpr int PER = (BM * BK) / NTH;  // complex elements per thread per operand
  c2 ra[PER], rb[PER];

  auto load = [&](int k0, int kend) {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = tid + it * NTH;
      int m, k;
      if (!TA) { m = idx / BK; k = idx % BK; } else { k = idx / BM; m = idx % BM; }
      const int gm = m0 + m, gk = k0 + k;
      c2 v;
      v.x = T(0); v.y = T(0);
      // rows outside the sub-block are not needed (their products are not stored)
      if (gm < M && gk < kend && m >= job.r0 && m < job.r1)
        v = TA ? Ab[(long long)gk * lda + gm] : Ab[(long long)gm * lda + gk];
      if (CA) v.y = -v.y;
      ra[it] = v;
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = tid + it * NTH;
      int n, k;
      if (!TB) { k = idx / BN; n = idx % BN; } else { n = idx / BK; k = idx % BK; }
      const int gn = n0 + n, gk = k0 + k;
      c2 v;
      v.x = T(0); v.y = T(0);
      if (gn < N && gk < kend && n >= job.c0 && n < job.c1)
        v = TB ? Bb[(long long)gn * ldb + gk] : Bb[(long long)gk * ldb + gn];
      if (CB) v.y = -v.y;
      rb[it] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = tid + it * NTH;
      int m, k;
      if (!TA) { m = idx / BK; k = idx % BK; } else { k = idx / BM; m = idx % BM; }
      As_r[buf][k][m] = ra[it].x;
      As_i[buf][k][m] = ra[it].y;
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = tid + it * NTH;
      int n, k;
      if (!TB) { k = idx / BN; n = idx % BN; } else { n = idx / BK; k = idx % BK; }
      Bs_r[buf][k][n] = rb[it].x;
      Bs_i[buf][k][n] = rb[it].y;
    }
  };

  // Three real products per complex multiply-add (the 3M form):
  // p1 = sum ar br, p2 = sum ai bi, p3 = sum (ar + ai)(br + bi); then
  // Re = p1 - p2 and Im = p3 - p1 - p2.  The operand sums are formed in
  // registers after the LDS reads, so the matrix cores issue 3/4 of the
  // products of the four-product form at the same LDS traffic.
  acc_t p1[SI][SJ], p2[SI][SJ], p3[SI][SJ];
#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j) {
      p1[i][j] = acc_t{0, 0, 0, 0};
      p2[i][j] = acc_t{0, 0, 0, 0};
      p3[i][j] = acc_t{0, 0, 0, 0};
    }

  const int lr = lane & 15, lk = lane >> 4;
  // the wave's 16 x 16 pieces that meet the sub-block (the others skip their
  // products and are not stored)
  bool act_i[SI], act_j[SJ];
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    const int r = wm * (BM / WM) + i * 16;
    act_i[i] = r < job.r1 && r + 16 > job.r0;
  }
#pragma unroll
  for (int j = 0; j < SJ; ++j) {
    const int c = wn * (BN / WN) + j * 16;
    act_j[j] = c < job.c1 && c + 16 > job.c0;
  }
  // The wave's piece rows ro[i] and columns co[j] (tile offsets) and which
  // of its pieces it computes.  By quadrant, a sub-block covering part of the
  // tile can leave some waves with four pieces and others with none, and the
  // item lasts as long as its busiest wave.  With four waves of 2 x 2 pieces,
  // a block-sparse item whose covered pieces (ni x nj of 16 x 16) number at
  // most four gets one per wave, one at most two pieces wide a row strip per
  // wave, one at most two pieces tall a column strip per wave; larger ones
  // keep the quadrants.
  int ro[SI], co[SJ];
  bool pact[SI][SJ];
#pragma unroll
  for (int i = 0; i < SI; ++i) ro[i] = wm * (BM / WM) + i * 16;
#pragma unroll
  for (int j = 0; j < SJ; ++j) co[j] = wn * (BN / WN) + j * 16;
#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j) pact[i][j] = act_i[i] && act_j[j];
  if constexpr (SI == 2 && SJ == 2 && WM * WN == 4) {
    const int pi0 = job.r0 >> 4, pj0 = job.c0 >> 4;
    const int ni = ((job.r1 + 15) >> 4) - pi0, nj = ((job.c1 + 15) >> 4) - pj0;
    const int shape = kit == nullptr ? 0 : ni * nj <= 4 ? 1 : nj <= 2 ? 2 : ni <= 2 ? 3 : 0;
    if (shape != 0) {
#pragma unroll
      for (int i = 0; i < SI; ++i)
#pragma unroll
        for (int j = 0; j < SJ; ++j) pact[i][j] = false;
      ro[1] = ro[0] = 0;
      co[1] = co[0] = 0;
      if (shape == 1) {   // one piece per wave
        if (wave < ni * nj) {
          ro[0] = (pi0 + wave / nj) * 16;
          co[0] = (pj0 + wave % nj) * 16;
          pact[0][0] = true;
        }
      } else if (shape == 2) {   // row strips: row pi0 + wave, nj <= 2 pieces
        if (wave < ni) {
          ro[0] = (pi0 + wave) * 16;
#pragma unroll
          for (int j = 0; j < SJ; ++j) {
            co[j] = (pj0 + (j < nj ? j : 0)) * 16;
            pact[0][j] = j < nj;
          }
        }
      } else {   // column strips: column pj0 + wave, ni <= 2 pieces
        if (wave < nj) {
          co[0] = (pj0 + wave) * 16;
#pragma unroll
          for (int i = 0; i < SI; ++i) {
            ro[i] = (pi0 + (i < ni ? i : 0)) * 16;
            pact[i][0] = i < ni;
          }
        }
      }
    }
  }
  // double-buffered LDS: compute on `cur` while the next tile's global loads
  // are in flight, then store them into the other buffer; one barrier per
  // tile.  The K steps walk the tile's intervals in order.
  const KIter kr_ = job.kr;
  int iv = 0, k0 = 0, kend = 0;
  if (kr_.n > 0) {
    const int2 I0 = kr_.at(0);
    k0 = I0.x;
    kend = I0.y;
    load(k0, kend);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (bool go = kr_.n > 0; go;) {
    int nk0 = k0 + BK, nkend = kend, niv = iv;
    if (nk0 >= kend) {
      ++niv;
      if (niv < kr_.n) {
        const int2 J = kr_.at(niv);
        nk0 = J.x;
        nkend = J.y;
      }
    }
    const bool more = niv < kr_.n;
    if (more) load(nk0, nkend);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      // the stage's entries past the interval end are zeros: skip their
      // MFMA steps (K intervals of charge blocks end anywhere)
      if (kk > 0 && k0 + kk >= kend) break;
      const int kr = kk + lk;
      T a_r[SI], a_i[SI], a_s[SI], b_r[SJ], b_i[SJ], b_s[SJ];
#pragma unroll
      for (int i = 0; i < SI; ++i) {
        a_r[i] = As_r[cur][kr][ro[i] + lr];
        a_i[i] = As_i[cur][kr][ro[i] + lr];
        a_s[i] = a_r[i] + a_i[i];
      }
#pragma unroll
      for (int j = 0; j < SJ; ++j) {
        b_r[j] = Bs_r[cur][kr][co[j] + lr];
        b_i[j] = Bs_i[cur][kr][co[j] + lr];
        b_s[j] = b_r[j] + b_i[j];
      }
#pragma unroll
      for (int i = 0; i < SI; ++i)
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
          if (!pact[i][j]) continue;
          p1[i][j] = mfma(a_r[i], b_r[j], p1[i][j]);
          p2[i][j] = mfma(a_i[i], b_i[j], p2[i][j]);
          p3[i][j] = mfma(a_s[i], b_s[j], p3[i][j]);
        }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
    go = more;
    iv = niv;
    k0 = nk0;
    kend = nkend;
  }

  const bool has_beta = (br != T(0)) || (bi != T(0));
#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // output row inside the 16x16 tile: the f32 MFMA puts rows 4*(lane/16)+r
        // in a lane, the f64 MFMA rows (lane/16)+4*r (columns are lane%16 for both)
        if (!pact[i][j]) continue;
        const int tr = sizeof(T) == 8 ? (lk + 4 * r) : (lk * 4 + r);
        const int lm = ro[i] + tr, ln = co[j] + lr;
        const int gm = m0 + lm;
        const int gn = n0 + ln;
        if (gm < M && gn < N && lm >= job.r0 && lm < job.r1 && ln >= job.c0 && ln < job.c1) {
          const T q1 = p1[i][j][r], q2 = p2[i][j][r];
          const T xr = q1 - q2, xi = p3[i][j][r] - q1 - q2;
          c2 o;
          o.x = ar * xr - ai * xi;
          o.y = ar * xi + ai * xr;
          if (has_beta) {
            const c2 old = Cb[(long long)gm * ldc + gn];
            o.x += br * old.x - bi * old.y;
            o.y += br * old.y + bi * old.x;
          }
          Cb[(long long)gm * ldc + gn] = o;
        }
      }
}

// ---------------------------------------------------------------- BF16 GEMM
// Complex GEMM on complex64 operands with BF16 MFMA inputs and FP32
// accumulation (v_mfma_f32_16x16x32_bf16: lane l holds row l%16 and the
// eight k values 8*(l/16)..+7 of its operand; outputs as the f32 MFMA).
// Operand tiles are rounded to BF16 (nearest even) as they are staged into
// LDS, one plane per real/imaginary part, k contiguous.  SPLIT = 1 keeps the
// rounding residual as a second BF16 term, x = hi + lo, and forms each real
// product as ah bh + ah bl + al bh (three MFMA products, ~16-bit operands).
constexpr int BK2 = 32, BKP2 = BK2 + 8, PL2 = 64 * BKP2;

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

typedef unsigned short us4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ inline f4 mfma_bf16(uint4 a, uint4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                  0);
}
__device__ inline uint4 bf16_neg(uint4 v) {
  const unsigned s = 0x80008000u;
  return uint4{v.x ^ s, v.y ^ s, v.z ^ s, v.w ^ s};
}

// A ROWS x 32 complex operand tile (rows r = m of A or n of B) as ROWS/32
// quads of four consecutive k per thread.  KC: k is the contiguous index in
// memory.  Planes (real, imaginary; and the residual terms with SPLIT) of
// ROWS x BKP2 bf16 each, k contiguous.
// (rows lo .. hi of the tile only: the others are not needed)
template <bool KC, bool CONJ, int ROWS = 64>
__device__ inline void bf_load(const float2* __restrict__ X, long long ld, int r0, int R, int k0, int ke, int tid,
                               float2 (&v)[ROWS / 32][4], int lo = 0, int hi = ROWS) {
#pragma unroll
  for (int it = 0; it < ROWS / 32; ++it) {
    const int q = tid + it * NT;
    const int row = KC ? (q >> 3) : (q % ROWS);
    const int kq = KC ? (q & 7) : (q / ROWS);
    const int gr = r0 + row;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gk = k0 + 4 * kq + j;
      float2 e;
      e.x = 0.f;
      e.y = 0.f;
      if (gr < R && gk < ke && row >= lo && row < hi) e = KC ? X[(long long)gr * ld + gk] : X[(long long)gk * ld + gr];
      if (CONJ) e.y = -e.y;
      v[it][j] = e;
    }
  }
}

template <bool KC, int SPLIT, int ROWS = 64>
__device__ inline void bf_store(unsigned short* P, int tid, const float2 (&v)[ROWS / 32][4]) {
  constexpr int PL = ROWS * BKP2;
#pragma unroll
  for (int it = 0; it < ROWS / 32; ++it) {
    const int q = tid + it * NT;
    const int row = KC ? (q >> 3) : (q % ROWS);
    const int kq = KC ? (q & 7) : (q / ROWS);
    us4 hr, hi, lr, li;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      hr[j] = bf16_rne(v[it][j].x);
      hi[j] = bf16_rne(v[it][j].y);
      if (SPLIT) {
        lr[j] = bf16_rne(v[it][j].x - bf16_val(hr[j]));
        li[j] = bf16_rne(v[it][j].y - bf16_val(hi[j]));
      }
    }
    const int off = row * BKP2 + 4 * kq;
    *reinterpret_cast<us4*>(P + off) = hr;
    *reinterpret_cast<us4*>(P + PL + off) = hi;
    if (SPLIT) {
      *reinterpret_cast<us4*>(P + 2 * PL + off) = lr;
      *reinterpret_cast<us4*>(P + 3 * PL + off) = li;
    }
  }
}

template <int SPLIT, bool TA, bool CA, bool TB, bool CB, int TAG>
__global__ __launch_bounds__(NT) void gemm_bf16_kernel(int M, int N, int K, float ar, float ai,
                                                        const float* __restrict__ A, long long lda, long long sa,
                                                        const float* __restrict__ B, long long ldb, long long sb,
                                                        float br, float bi, float* __restrict__ C, long long ldc,
                                                        long long sc, int S, int Kc, long long sps,
                                                        const int4* __restrict__ kit, const int2* __restrict__ kiv) {
  constexpr int NPL = SPLIT ? 4 : 2;
  __shared__ __attribute__((aligned(16))) unsigned short As[2][NPL * PL2];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NPL * PL2];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const TileJob job = tile_job(M, N, K, S, Kc, kit, kiv);
  const int m0 = job.m0, n0 = job.n0, split = job.split;
  const long long bz = job.bz;
  const float2* Ab = reinterpret_cast<const float2*>(A) + bz * sa;
  const float2* Bb = reinterpret_cast<const float2*>(B) + bz * sb;
  float2* Cb = reinterpret_cast<float2*>(C) + bz * sc + split * sps;

  // A tile rows are m (k contiguous when A is not transposed); B tile rows
  // are n (k contiguous when B is transposed)
  float2 va[2][4], vb[2][4];
  auto load = [&](int k0, int kend) {
    bf_load<!TA, CA>(Ab, lda, m0, M, k0, kend, tid, va, job.r0, job.r1);
    bf_load<TB, CB>(Bb, ldb, n0, N, k0, kend, tid, vb, job.c0, job.c1);
  };
  auto store = [&](int buf) {
    bf_store<!TA, SPLIT>(As[buf], tid, va);
    bf_store<TB, SPLIT>(Bs[buf], tid, vb);
  };

  f4 cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = f4{0, 0, 0, 0};
      ci[i][j] = f4{0, 0, 0, 0};
    }

  const int lr = lane & 15, lk = lane >> 4;
  bool act_i[2], act_j[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r = wm * 32 + i * 16, c = wn * 32 + i * 16;
    act_i[i] = r < job.r1 && r + 16 > job.r0;
    act_j[i] = c < job.c1 && c + 16 > job.c0;
  }
  const KIter kr_ = job.kr;
  int iv = 0, k0 = 0, kend = 0;
  if (kr_.n > 0) {
    const int2 I0 = kr_.at(0);
    k0 = I0.x;
    kend = I0.y;
    load(k0, kend);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (bool go = kr_.n > 0; go;) {
    int nk0 = k0 + BK2, nkend = kend, niv = iv;
    if (nk0 >= kend) {
      ++niv;
      if (niv < kr_.n) {
        const int2 J = kr_.at(niv);
        nk0 = J.x;
        nkend = J.y;
      }
    }
    const bool more = niv < kr_.n;
    if (more) load(nk0, nkend);
    const unsigned short* Ap = As[cur];
    const unsigned short* Bp = Bs[cur];
    uint4 a_hr[2], a_hi[2], a_lr[2], a_li[2], b_hr[2], b_hi[2], b_hn[2], b_lr[2], b_li[2], b_ln[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int off = (wm * 32 + i * 16 + lr) * BKP2 + 8 * lk;
      a_hr[i] = *reinterpret_cast<const uint4*>(Ap + off);
      a_hi[i] = *reinterpret_cast<const uint4*>(Ap + PL2 + off);
      if (SPLIT) {
        a_lr[i] = *reinterpret_cast<const uint4*>(Ap + 2 * PL2 + off);
        a_li[i] = *reinterpret_cast<const uint4*>(Ap + 3 * PL2 + off);
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int off = (wn * 32 + j * 16 + lr) * BKP2 + 8 * lk;
      b_hr[j] = *reinterpret_cast<const uint4*>(Bp + off);
      b_hi[j] = *reinterpret_cast<const uint4*>(Bp + PL2 + off);
      b_hn[j] = bf16_neg(b_hi[j]);
      if (SPLIT) {
        b_lr[j] = *reinterpret_cast<const uint4*>(Bp + 2 * PL2 + off);
        b_li[j] = *reinterpret_cast<const uint4*>(Bp + 3 * PL2 + off);
        b_ln[j] = bf16_neg(b_li[j]);
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (!(act_i[i] && act_j[j])) continue;
        if (SPLIT) {
          cr[i][j] = mfma_bf16(a_hr[i], b_lr[j], cr[i][j]);
          cr[i][j] = mfma_bf16(a_lr[i], b_hr[j], cr[i][j]);
          cr[i][j] = mfma_bf16(a_hi[i], b_ln[j], cr[i][j]);
          cr[i][j] = mfma_bf16(a_li[i], b_hn[j], cr[i][j]);
          ci[i][j] = mfma_bf16(a_hr[i], b_li[j], ci[i][j]);
          ci[i][j] = mfma_bf16(a_lr[i], b_hi[j], ci[i][j]);
          ci[i][j] = mfma_bf16(a_hi[i], b_lr[j], ci[i][j]);
          ci[i][j] = mfma_bf16(a_li[i], b_hr[j], ci[i][j]);
        }
        cr[i][j] = mfma_bf16(a_hr[i], b_hr[j], cr[i][j]);
        cr[i][j] = mfma_bf16(a_hi[i], b_hn[j], cr[i][j]);
        ci[i][j] = mfma_bf16(a_hr[i], b_hi[j], ci[i][j]);
        ci[i][j] = mfma_bf16(a_hi[i], b_hr[j], ci[i][j]);
      }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
    go = more;
    iv = niv;
    k0 = nk0;
    kend = nkend;
  }

  const bool has_beta = (br != 0.f) || (bi != 0.f);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lm = wm * 32 + i * 16 + lk * 4 + r, ln = wn * 32 + j * 16 + lr;
        const int gm = m0 + lm;
        const int gn = n0 + ln;
        if (gm < M && gn < N && lm >= job.r0 && lm < job.r1 && ln >= job.c0 && ln < job.c1) {
          const float xr = cr[i][j][r], xi = ci[i][j][r];
          float2 o;
          o.x = ar * xr - ai * xi;
          o.y = ar * xi + ai * xr;
          if (has_beta) {
            const float2 old = Cb[(long long)gm * ldc + gn];
            o.x += br * old.x - bi * old.y;
            o.y += br * old.y + bi * old.x;
          }
          Cb[(long long)gm * ldc + gn] = o;
        }
      }
}

// Deterministic split-K reduction: C = alpha * sum_s P[s] + beta * C.
template <typename T>
__global__ void splitk_reduce_kernel(const T* __restrict__ P, int S, long long M, long long N, T ar, T ai,
                                     T br, T bi, T* __restrict__ C, long long ldc) {
  using c2 = typename VT<T>::c2;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const c2* Pc = reinterpret_cast<const c2*>(P);
  T xr = T(0), xi = T(0);
  for (int s = 0; s < S; ++s) {
    const c2 v = Pc[(long long)s * M * N + idx];
    xr += v.x;
    xi += v.y;
  }
  const long long m = idx / N, n = idx % N;
  c2* Cc = reinterpret_cast<c2*>(C);
  c2 o;
  o.x = ar * xr - ai * xi;
  o.y = ar * xi + ai * xr;
  if (br != T(0) || bi != T(0)) {
    const c2 old = Cc[m * ldc + n];
    o.x += br * old.x - bi * old.y;
    o.y += br * old.y + bi * old.x;
  }
  Cc[m * ldc + n] = o;
}

// Split-K reduction of a block-sparse product: C[b] = alpha * sum of the
// nonempty parts of each tile + beta * C[b]; the parts are P[s][b][m][n].
template <typename T>
__global__ void splitk_reduce_map_kernel(const T* __restrict__ P, int batch, long long M, long long N, int gx,
                                         const int* __restrict__ tinfo, T ar, T ai, T br, T bi, T* __restrict__ C,
                                         long long ldc, long long sc) {
  using c2 = typename VT<T>::c2;
  const long long MN = M * N;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= MN * batch) return;
  const long long b = idx / MN, r = idx % MN, m = r / N, n = r % N;
  const long long tiles = ((M + BM - 1) / BM) * (long long)gx;
  const int* ti = tinfo + 6 * (b * tiles + (m / BM) * gx + n / BN);
  const int ns = ti[2 + ((m % BM) >= ti[0] ? 2 : 0) + ((n % BN) >= ti[1] ? 1 : 0)];
  const c2* Pc = reinterpret_cast<const c2*>(P);
  T xr = T(0), xi = T(0);
  for (int s = 0; s < ns; ++s) {
    const c2 v = Pc[(long long)s * batch * MN + idx];
    xr += v.x;
    xi += v.y;
  }
  c2* Cc = reinterpret_cast<c2*>(C) + b * sc + m * ldc + n;
  c2 o;
  o.x = ar * xr - ai * xi;
  o.y = ar * xi + ai * xr;
  if (br != T(0) || bi != T(0)) {
    const c2 old = *Cc;
    o.x += br * old.x - bi * old.y;
    o.y += br * old.y + bi * old.x;
  }
  *Cc = o;
}

// Number of K splits: about one workgroup per CU when the output has few
// tiles (Gram matrices, back transformations: 16-64 tiles would leave most
// of the 256 CUs idle), each split keeping >= 64 of K.  The partial products
// (S M N complex) mostly stay in the last-level cache.
inline int choose_splits(int M, int N, int K, int batch, size_t ws_bytes, size_t cbytes) {
  const long long tiles = (long long)((M + BM - 1) / BM) * ((N + BN - 1) / BN) * batch;
  if (batch != 1 || ws_bytes == 0 || tiles >= 256 || K < 128) return 1;
  int S = (int)std::min<long long>((256 + tiles - 1) / tiles, K / 64);
  S = std::min(S, 32);
  while (S > 1 && (size_t)S * M * N * cbytes > ws_bytes) --S;
  return std::max(S, 1);
}

// Compute mode of the complex64 GEMMs on the calling host thread:
// 0 FP32 MFMA, 1 BF16 MFMA, 2 three-term BF16 split (see gemm_bf16_kernel).
thread_local int tl_float_mode = 0;

// block-sparse map of the next product issued from the calling host thread
thread_local const kern::KMap* tl_kmap = nullptr;

template <typename T, int MODE, bool TA, bool CA, bool TB, bool CB, int TAG>
void launch_tiles(dim3 grid, hipStream_t s, int M, int N, int K, T ar, T ai, const T* A, long long lda,
                  long long sa, const T* B, long long ldb, long long sb, T br, T bi, T* C, long long ldc,
                  long long sc, int S, int Kc, long long sps, const int4* kit = nullptr, const int2* kiv = nullptr) {
  if constexpr (MODE == 0) {
    hipLaunchKernelGGL((gemm_kernel<T, TA, CA, TB, CB, TAG>), grid, dim3(gemm_threads<T>()), 0, s, M, N, K, ar, ai, A,
                       lda, sa, B, ldb, sb, br, bi, C, ldc, sc, S, Kc, sps, kit, kiv);
  } else {
    hipLaunchKernelGGL((gemm_bf16_kernel<MODE - 1, TA, CA, TB, CB, TAG>), grid, dim3(NT), 0, s, M, N, K, ar, ai,
                       A, lda, sa, B, ldb, sb, br, bi, C, ldc, sc, S, Kc, sps, kit, kiv);
  }
}

template <typename T, int MODE, int OA, int OB, int TAG>
void launch_gemm_mode(hipStream_t s, int M, int N, int K, zc alpha, const void* A, long long lda, long long sa,
                      const void* B, long long ldb, long long sb, zc beta, void* C, long long ldc, long long sc,
                      int batch, void* ws, size_t ws_bytes) {
  constexpr bool TA = (OA == TDVP_OP_T || OA == TDVP_OP_C), CA = (OA == TDVP_OP_C || OA == TDVP_OP_R);
  constexpr bool TB = (OB == TDVP_OP_T || OB == TDVP_OP_C), CB = (OB == TDVP_OP_C || OB == TDVP_OP_R);
  constexpr int KSTEP = MODE == 0 ? BK : BK2;
  const T* a = static_cast<const T*>(A);
  const T* b = static_cast<const T*>(B);
  const kern::KMap* km = tl_kmap;
  if (km && km->batch == batch) {
    if (km->M != M || km->N != N || km->K != K) TDVP_THROW(TDVP_ERR_ARG, "block-sparse map does not fit the product");
    const int gx = (N + BN - 1) / BN;
    if (km->splits > 1) {
      using c2 = typename VT<T>::c2;
      const long long MN = (long long)M * N;
      if (!km->part || km->part_bytes < (size_t)km->splits * batch * MN * sizeof(c2))
        TDVP_THROW(TDVP_ERR_ARG, "block-sparse map without room for its partial products");
      T* P = static_cast<T*>(km->part);
      if (km->n_items > 0)
        launch_tiles<T, MODE, TA, CA, TB, CB, TAG>(dim3(km->n_items), s, M, N, K, T(1), T(0), a, lda, sa, b, ldb, sb,
                                                   T(0), T(0), P, (long long)N, MN, km->splits, std::max(K, 1),
                                                   MN * batch, km->items, reinterpret_cast<const int2*>(km->iv));
      hipLaunchKernelGGL(splitk_reduce_map_kernel<T>, dim3((unsigned)((MN * batch + 255) / 256)), dim3(256), 0, s, P,
                         batch, (long long)M, (long long)N, gx, km->tinfo, T(alpha.real()), T(alpha.imag()),
                         T(beta.real()), T(beta.imag()), static_cast<T*>(C), ldc, sc);
      return;
    }
    if (!km->partial && km->n_items < batch * gx * ((M + BM - 1) / BM))
      TDVP_THROW(TDVP_ERR_ARG, "block-sparse map without every tile");
    if (km->n_items == 0) return;   // a partial map with nothing to write
    launch_tiles<T, MODE, TA, CA, TB, CB, TAG>(dim3(km->n_items), s, M, N, K, T(alpha.real()), T(alpha.imag()), a,
                                               lda, sa, b, ldb, sb, T(beta.real()), T(beta.imag()),
                                               static_cast<T*>(C), ldc, sc, 1, std::max(K, 1), 0LL, km->items,
                                               reinterpret_cast<const int2*>(km->iv));
    return;
  }
  const int S = choose_splits(M, N, K, batch, ws_bytes, sizeof(typename VT<T>::c2));
  if (S == 1) {
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
    launch_tiles<T, MODE, TA, CA, TB, CB, TAG>(grid, s, M, N, K, T(alpha.real()), T(alpha.imag()), a, lda, sa, b,
                                               ldb, sb, T(beta.real()), T(beta.imag()), static_cast<T*>(C), ldc,
                                               sc, 1, std::max(K, 1), 0LL);
    return;
  }
  const int Kc = ((K + S - 1) / S + KSTEP - 1) / KSTEP * KSTEP;
  const int Sx = (K + Kc - 1) / Kc;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, Sx);
  launch_tiles<T, MODE, TA, CA, TB, CB, TAG>(grid, s, M, N, K, T(1), T(0), a, lda, sa, b, ldb, sb, T(0), T(0),
                                             static_cast<T*>(ws), (long long)N, 0LL, Sx, Kc, (long long)M * N);
  const long long MN = (long long)M * N;
  hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, s,
                     static_cast<const T*>(ws), Sx, (long long)M, (long long)N, T(alpha.real()), T(alpha.imag()),
                     T(beta.real()), T(beta.imag()), static_cast<T*>(C), ldc);
}

template <typename T, int OA, int OB, int TAG = 0>
void launch_gemm(hipStream_t s, int M, int N, int K, zc alpha, const void* A, long long lda,
                 long long sa, const void* B, long long ldb, long long sb, zc beta, void* C,
                 long long ldc, long long sc, int batch, void* ws = nullptr, size_t ws_bytes = 0) {
  if constexpr (sizeof(T) == 4) {
    if (tl_float_mode == 1) {
      launch_gemm_mode<T, 1, OA, OB, TAG>(s, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws,
                                          ws_bytes);
      return;
    }
    if (tl_float_mode == 2) {
      launch_gemm_mode<T, 2, OA, OB, TAG>(s, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws,
                                          ws_bytes);
      return;
    }
  }
  launch_gemm_mode<T, 0, OA, OB, TAG>(s, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws,
                                      ws_bytes);
}

template <typename T, int OA>
void dispatch_b(hipStream_t s, int opb, int M, int N, int K, zc alpha, const void* A, long long lda,
                long long sa, const void* B, long long ldb, long long sb, zc beta, void* C,
                long long ldc, long long sc, int batch, void* ws, size_t wsb) {
  switch (opb) {
    case TDVP_OP_N: launch_gemm<T, OA, TDVP_OP_N>(s, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws, wsb); break;
    case TDVP_OP_T: launch_gemm<T, OA, TDVP_OP_T>(s, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws, wsb); break;
    case TDVP_OP_C: launch_gemm<T, OA, TDVP_OP_C>(s, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws, wsb); break;
    case TDVP_OP_R: launch_gemm<T, OA, TDVP_OP_R>(s, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws, wsb); break;
    default: TDVP_THROW(TDVP_ERR_ARG, "bad GEMM op_b");
  }
}

// ---------------------------------------------------------------- W apply
constexpr int WQ = 64;      // q extent per block
constexpr int WNT = 256;
constexpr int WMAX_CH = 256;   // channels (MPO index x physical index) of a charged stage

template <typename T>
__global__ __launch_bounds__(WNT) void wapply_kernel(const T* __restrict__ in, T* __restrict__ out, long long nQ,
                                                      long long isP, long long isQ, long long is1,
                                                      long long is2, long long osP, long long osQ,
                                                      long long os1, long long os2,
                                                      const int* __restrict__ rowptr,
                                                      const int* __restrict__ col,
                                                      const double2* __restrict__ val, int n_in,
                                                      int n_out, kern::WCharges wc) {
  using c2 = typename VT<T>::c2;
  extern __shared__ unsigned char smem_raw[];
  c2* lds = reinterpret_cast<c2*>(smem_raw);  // [n_in][WQ]
  // charge difference of each column of the block and the channels' own
  // (charged contractions only)
  __shared__ int dq[WQ];
  __shared__ int din_s[WMAX_CH], dout_s[WMAX_CH];
  const long long p = blockIdx.y;
  const long long q0 = (long long)blockIdx.x * WQ;
  const c2* inb = reinterpret_cast<const c2*>(in);
  c2* outb = reinterpret_cast<c2*>(out);
  const bool charged = wc.ql != nullptr;
  if (charged) {
    for (int t = threadIdx.x; t < WQ; t += WNT) dq[t] = q0 + t < nQ ? wc.qr[q0 + t] - wc.ql[p] : 0;
    for (int t = threadIdx.x; t < n_in; t += WNT) din_s[t] = wc.din[t];
    for (int t = threadIdx.x; t < n_out; t += WNT) dout_s[t] = wc.dout[t];
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < n_in * WQ; idx += WNT) {
    const int c = idx / WQ, q = idx % WQ;
    c2 v;
    v.x = T(0); v.y = T(0);
    if (q0 + q < nQ && (!charged || din_s[c] == dq[q]))
      v = inb[p * isP + (q0 + q) * isQ + (c >> 1) * is1 + (c & 1) * is2];
    lds[idx] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n_out * WQ; idx += WNT) {
    const int o = idx / WQ, q = idx % WQ;
    if (q0 + q >= nQ) continue;
    T sr = T(0), si = T(0);
    // an output of another charge is an exact zero (+0, as the sum of the
    // zero inputs would give), stored unless the output already holds it
    const bool zero = charged && dout_s[o] != dq[q];
    if (zero && wc.zeros_kept) continue;
    const int e_end = zero ? rowptr[o] : rowptr[o + 1];
    for (int e = rowptr[o]; e < e_end; ++e) {
      const double2 w = val[e];
      const c2 x = lds[col[e] * WQ + q];
      sr += T(w.x) * x.x - T(w.y) * x.y;
      si += T(w.x) * x.y + T(w.y) * x.x;
    }
    c2 r;
    r.x = sr;
    r.y = si;
    outb[p * osP + (q0 + q) * osQ + (o >> 1) * os1 + (o & 1) * os2] = r;
  }
}

// ---------------------------------------------------------------- vectors
constexpr int VNT = 256;
constexpr int DOT_CHUNK = 1024;

// sum over the wave (all 64 lanes active; every lane gets the total)
__device__ inline double warp_sum(double v) { return wave::sum(v); }

__device__ inline double block_sum(double v, double* sh) {
  v = warp_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < VNT / 64; ++i) t += sh[i];
  return t;  // valid on thread 0
}

// One block per (vector j, chunk): partial[b * nv + j] = sum over the chunk.
template <bool CONJ>
__global__ __launch_bounds__(VNT) void zdots_partial_kernel(const double2* __restrict__ V, long long ldv, int nv,
                                                             const double2* __restrict__ w, long long n,
                                                             double2* __restrict__ partial) {
  __shared__ double sh[VNT / 64];
  const int j = blockIdx.y;
  const long long beg = (long long)blockIdx.x * DOT_CHUNK;
  const long long end = min(n, beg + DOT_CHUNK);
  double sr = 0.0, si = 0.0;
  const double2* v = V + (long long)j * ldv;
  for (long long x = beg + threadIdx.x; x < end; x += VNT) {
    const double2 a = v[x], b = w[x];
    if (CONJ) {                    // conj(a) * b
      sr += a.x * b.x + a.y * b.y;
      si += a.x * b.y - a.y * b.x;
    } else {                       // a * b
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
  }
  const double tr = block_sum(sr, sh);
  const double ti = block_sum(si, sh);
  if (threadIdx.x == 0) partial[(long long)blockIdx.x * nv + j] = make_double2(tr, ti);
}

// one block per vector: out[j] = sum over the blocks' partials (fixed tree)
__global__ __launch_bounds__(VNT) void zdots_final_kernel(const double2* __restrict__ partial, int nb, int nv,
                                                           double2* __restrict__ out) {
  __shared__ double sh[VNT / 64];
  const int j = blockIdx.x;
  double sr = 0.0, si = 0.0;
  for (int b = threadIdx.x; b < nb; b += VNT) {
    const double2 p = partial[(long long)b * nv + j];
    sr += p.x;
    si += p.y;
  }
  const double tr = block_sum(sr, sh);
  const double ti = block_sum(si, sh);
  if (threadIdx.x == 0) out[j] = make_double2(tr, ti);
}

__global__ __launch_bounds__(VNT) void zcombine_kernel(double2* __restrict__ w, const double2* __restrict__ V,
                                                        long long ldv, int nv, const double2* __restrict__ c,
                                                        double sign, long long n) {
  const long long x = (long long)blockIdx.x * VNT + threadIdx.x;
  if (x >= n) return;
  double sr = 0.0, si = 0.0;
  for (int j = 0; j < nv; ++j) {
    const double2 cj = c[j];
    const double2 v = V[(long long)j * ldv + x];
    sr += cj.x * v.x - cj.y * v.y;
    si += cj.x * v.y + cj.y * v.x;
  }
  double2 o = w[x];
  o.x += sign * sr;
  o.y += sign * si;
  w[x] = o;
}

__global__ void zscale_kernel(double2* __restrict__ dst, const double2* __restrict__ src, double ar,
                              double ai, long long n) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const double2 v = src[x];
  dst[x] = make_double2(ar * v.x - ai * v.y, ar * v.y + ai * v.x);
}

// dst = src / sqrt(Re *nrm2): normalisation by a norm that is still on the device
// w += sign * V c with c_j the sum of the nb partial dot products
// partial[b * nv + j] (zdots_partial_kernel's layout): every block forms c
// itself, in the same fixed order, so no separate reduction launch is
// needed; block 0 also stores c in cout.  With NORM, the block's partial sum
// of |w|^2 goes to npart.
constexpr int ZC_MAXV = 64;
template <bool NORM>
__global__ __launch_bounds__(VNT) void zcombine_p_kernel(double2* __restrict__ w, const double2* __restrict__ V,
                                                         long long ldv, int nv, const double2* __restrict__ partial,
                                                         int nb, double sign, long long n, double2* __restrict__ cout,
                                                         double2* __restrict__ npart) {
  __shared__ double2 sc[ZC_MAXV];
  __shared__ double sh[VNT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = wv; j < nv; j += VNT / 64) {
    double re = 0.0, im = 0.0;
    for (int b = lane; b < nb; b += 64) {
      const double2 p = partial[(long long)b * nv + j];
      re += p.x;
      im += p.y;
    }
    re = warp_sum(re);
    im = warp_sum(im);
    if (lane == 0) sc[j] = make_double2(re, im);
  }
  __syncthreads();
  if (blockIdx.x == 0 && cout)
    for (int j = threadIdx.x; j < nv; j += VNT) cout[j] = sc[j];
  const long long x = (long long)blockIdx.x * VNT + threadIdx.x;
  double sq = 0.0;
  if (x < n) {
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < nv; ++j) {
      const double2 cj = sc[j];
      const double2 v = V[(long long)j * ldv + x];
      sr += cj.x * v.x - cj.y * v.y;
      si += cj.x * v.y + cj.y * v.x;
    }
    double2 o = w[x];
    o.x += sign * sr;
    o.y += sign * si;
    w[x] = o;
    sq = o.x * o.x + o.y * o.y;
  }
  if (NORM) {
    const double t = block_sum(sq, sh);
    if (threadIdx.x == 0) npart[blockIdx.x] = make_double2(t, 0.0);
  }
}

// The same update, then the block's partial dot products of the updated w
// with every vector, dpart[blockIdx.x * nv + j] = sum over the block's x of
// conj(V[j][x]) w[x] (the layout zcombine_p_kernel reads): the second
// Gram-Schmidt pass gets its projections without another read of V.
__global__ __launch_bounds__(VNT) void zcombine_dots_kernel(double2* __restrict__ w, const double2* __restrict__ V,
                                                            long long ldv, int nv,
                                                            const double2* __restrict__ partial, int nb,
                                                            double sign, long long n, double2* __restrict__ cout,
                                                            double2* __restrict__ dpart) {
  __shared__ double2 sc[ZC_MAXV];
  __shared__ double2 sd[VNT / 64][ZC_MAXV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = wv; j < nv; j += VNT / 64) {
    double re = 0.0, im = 0.0;
    for (int b = lane; b < nb; b += 64) {
      const double2 p = partial[(long long)b * nv + j];
      re += p.x;
      im += p.y;
    }
    re = warp_sum(re);
    im = warp_sum(im);
    if (lane == 0) sc[j] = make_double2(re, im);
  }
  __syncthreads();
  if (blockIdx.x == 0 && cout)
    for (int j = threadIdx.x; j < nv; j += VNT) cout[j] = sc[j];
  const long long x = (long long)blockIdx.x * VNT + threadIdx.x;
  double2 o = make_double2(0.0, 0.0);
  if (x < n) {
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < nv; ++j) {
      const double2 cj = sc[j];
      const double2 v = V[(long long)j * ldv + x];
      sr += cj.x * v.x - cj.y * v.y;
      si += cj.x * v.y + cj.y * v.x;
    }
    o = w[x];
    o.x += sign * sr;
    o.y += sign * si;
    w[x] = o;
  }
  for (int j = 0; j < nv; ++j) {   // uniform loop: every lane takes part in the sums
    double re = 0.0, im = 0.0;
    if (x < n) {
      const double2 v = V[(long long)j * ldv + x];
      re = v.x * o.x + v.y * o.y;
      im = v.x * o.y - v.y * o.x;
    }
    re = warp_sum(re);
    im = warp_sum(im);
    if (lane == 0) sd[wv][j] = make_double2(re, im);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nv; j += VNT) {
    double2 t = sd[0][j];
#pragma unroll
    for (int q = 1; q < VNT / 64; ++q) {
      t.x += sd[q][j].x;
      t.y += sd[q][j].y;
    }
    dpart[(long long)blockIdx.x * nv + j] = t;
  }
}

// every block sums the np partial norms in the same fixed order, so all
// agree on |w|^2; block 0 also stores it
__global__ __launch_bounds__(VNT) void zscale_invnorm_kernel(double2* __restrict__ w,
                                                              const double2* __restrict__ partial, int np,
                                                              double2* __restrict__ out, long long n,
                                                              double2* host, const double2* __restrict__ coeffs,
                                                              int ncoef, int host_norm_at) {
  __shared__ double sh[VNT / 64];
  __shared__ double s_tot;
  double acc = 0.0;
  for (int b = threadIdx.x; b < np; b += VNT) acc += partial[b].x;
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    s_tot = t;
    if (blockIdx.x == 0) {
      out[0] = make_double2(t, 0.0);
      if (host) host[host_norm_at] = make_double2(t, 0.0);
    }
  }
  if (blockIdx.x == 0 && host)
    for (int j = threadIdx.x; j < ncoef; j += VNT) host[j] = coeffs[j];
  __syncthreads();
  const long long x = (long long)blockIdx.x * VNT + threadIdx.x;
  if (x >= n) return;
  const double inv = 1.0 / sqrt(fmax(s_tot, 0.0));
  const double2 v = w[x];
  w[x] = make_double2(v.x * inv, v.y * inv);
}

__global__ void z2c_kernel(float2* __restrict__ dst, const double2* __restrict__ src, long long n) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const double2 v = src[x];
  dst[x] = make_float2(float(v.x), float(v.y));
}

__global__ void c2z_kernel(double2* __restrict__ dst, const float2* __restrict__ src, long long n) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const float2 v = src[x];
  dst[x] = make_double2(double(v.x), double(v.y));
}

template <typename E>
__global__ void copy2d_kernel(E* __restrict__ dst, long long ldd, const E* __restrict__ src, long long lds,
                              long long rows, long long cols) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const long long i = idx / cols, j = idx % cols;
  dst[i * ldd + j] = src[i * lds + j];
}

__global__ void ztri_kernel(double2* __restrict__ dst, long long ldd, const double2* __restrict__ src,
                            long long lds, long long rows, long long cols, int mode) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const long long i = idx / cols, j = idx % cols;
  const bool keep = mode == 0 ? (j >= i) : (j <= i);
  dst[i * ldd + j] = keep ? src[i * lds + j] : make_double2(0.0, 0.0);
}

__global__ void zconjtrans_kernel(double2* __restrict__ dst, long long ldd, const double2* __restrict__ src,
                                  long long lds, long long rows, long long cols) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const long long i = idx / cols, j = idx % cols;
  const double2 v = src[j * lds + i];
  dst[i * ldd + j] = make_double2(v.x, -v.y);
}

// A = (S + S^H) / 2 (A may be S: each pair (i, j), j >= i, belongs to one
// thread); thread 0 also clears zero[0 .. nzero)
__global__ void zhermitize_kernel(double2* A, const double2* S, long long n, int* zero, int nzero) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx == 0)
    for (int k = 0; k < nzero; ++k) zero[k] = 0;
  if (idx >= n * n) return;
  const long long i = idx / n, j = idx % n;
  if (j < i) return;
  const double2 a = S[i * n + j], b = S[j * n + i];
  if (i == j) {
    A[i * n + j] = make_double2(a.x, 0.0);
  } else {
    const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    A[i * n + j] = h;
    A[j * n + i] = make_double2(h.x, -h.y);
  }
}

template <typename E>
__global__ void fill_kernel(E* __restrict__ dst, E v, long long n) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) dst[x] = v;
}

__global__ void zscale_phys_kernel(double2* __restrict__ G, long long nx, long long nq, double f0,
                                   double f1) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nx * 2 * nq) return;
  const long long s = (idx / nq) & 1;
  const double f = s ? f1 : f0;
  double2 v = G[idx];
  v.x *= f;
  v.y *= f;
  G[idx] = v;
}

__global__ void zscale_rc_kernel(double2* __restrict__ dst, long long ldd, const double2* __restrict__ src,
                                 long long lds, long long rows, long long cols, const double* __restrict__ f,
                                 int by_col) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const long long i = idx / cols, j = idx % cols;
  const double g = by_col ? f[j] : f[i];
  const double2 v = src[i * lds + j];
  dst[i * ldd + j] = make_double2(g * v.x, g * v.y);
}

__global__ void zshift_diag_kernel(double2* __restrict__ G, long long n, double a, double b) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  double2 v = G[idx];
  v.x *= a;
  v.y *= a;
  if (idx / n == idx % n) v.x += b;
  G[idx] = v;
}

// dst[i*ldd + j] = src[r(i)*lds + c(j)], r(i) = ridx ? ridx[i] : i, c likewise
__global__ void zgather_kernel(double2* __restrict__ dst, long long ldd, const double2* __restrict__ src,
                               long long lds, const int* __restrict__ ridx, long long nr,
                               const int* __restrict__ cidx, long long nc) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nr * nc) return;
  const long long i = idx / nc, j = idx % nc;
  const long long r = ridx ? ridx[i] : i, c = cidx ? cidx[j] : j;
  dst[i * ldd + j] = src[r * lds + c];
}

// dst[r(i)*ldd + c(j)] = src[i*lds + j], r(i) = ridx ? ridx[i] : i, c likewise
__global__ void zscatter_kernel(double2* __restrict__ dst, long long ldd, const double2* __restrict__ src,
                                long long lds, const int* __restrict__ ridx, long long nr,
                                const int* __restrict__ cidx, long long nc) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nr * nc) return;
  const long long i = idx / nc, j = idx % nc;
  const long long r = ridx ? ridx[i] : i, c = cidx ? cidx[j] : j;
  dst[r * ldd + c] = src[i * lds + j];
}

// dst[j] = H[idx[j]*n + idx[j]]; rows[pos[j]*n + idx[j]] = 1 (unit eigenvector of a 1 x 1 block)
template <typename D, typename S>
__device__ inline D cconv(S v) {
  D d;
  d.x = v.x;
  d.y = v.y;
  return d;
}
// block (x, r): entries x * 256 + t of row segment r
template <typename P, typename Dn, bool PACK>
__global__ void rows_pack_kernel(P* __restrict__ packed, Dn* __restrict__ dense, int rows, long long ld,
                                 const int* __restrict__ seg) {
  const int r = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int b0 = seg[r], len = seg[rows + r], off = seg[2 * rows + r];
  if (j >= len) return;
  if (PACK) packed[(long long)off + j] = cconv<P>(dense[(long long)r * ld + b0 + j]);
  else dense[(long long)r * ld + b0 + j] = cconv<Dn>(packed[(long long)off + j]);
}

// splitmix64 (Steele, Lea and Flood 2014) as a counter-based generator
__device__ inline unsigned long long mix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__global__ void zrandom_blocks_kernel(double2* __restrict__ E, int R, int C, const int* __restrict__ qr,
                                      const int* __restrict__ qc, unsigned long long seed) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)R * C) return;
  const int i = (int)(idx / C), j = (int)(idx % C);
  double2 v{0.0, 0.0};
  if (qr[i] == qc[j]) {
    const unsigned long long a = mix64(seed ^ (2ull * (unsigned long long)idx)),
                             b = mix64(seed ^ (2ull * (unsigned long long)idx + 1ull));
    v.x = (double)(a >> 11) * 0x1.0p-52 - 1.0;
    v.y = (double)(b >> 11) * 0x1.0p-52 - 1.0;
  }
  E[idx] = v;
}

__global__ void zunit_blocks_kernel(double2* __restrict__ dst, const double2* __restrict__ H, long long n,
                                    const int* __restrict__ idx, const int* __restrict__ pos, int cnt,
                                    double2* __restrict__ rows) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const long long i = idx[j];
  dst[j] = H[i * n + i];
  rows[(long long)pos[j] * n + i] = make_double2(1.0, 0.0);
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

namespace kern {

void set_float_mode(int mode) {
  if (mode < 0 || mode > 2) TDVP_THROW(TDVP_ERR_ARG, "bad complex64 GEMM mode");
  tl_float_mode = mode;
}
int float_mode() { return tl_float_mode; }

void set_kmap(const KMap* k) { tl_kmap = k; }
const KMap* current_kmap() { return tl_kmap; }

thread_local void* tl_split_ws = nullptr;
thread_local size_t tl_split_wsb = 0;
void set_split_workspace(void* p, size_t bytes) {
  tl_split_ws = p;
  tl_split_wsb = p ? bytes : 0;
}
SplitWorkspaceScope::SplitWorkspaceScope(void* p, size_t bytes) : saved_p(tl_split_ws), saved_b(tl_split_wsb) {
  set_split_workspace(p, bytes);
}
SplitWorkspaceScope::~SplitWorkspaceScope() { set_split_workspace(saved_p, saved_b); }

template <typename T>
void gemm(hipStream_t s, int opa, int opb, int M, int N, int K, zc alpha, const void* A, long long lda,
          long long sa, const void* B, long long ldb, long long sb, zc beta, void* C, long long ldc,
          long long sc, int batch, void* ws, size_t ws_bytes) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (!ws) {
    ws = tl_split_ws;
    ws_bytes = tl_split_wsb;
  }
  switch (opa) {
    case TDVP_OP_N: dispatch_b<T, TDVP_OP_N>(s, opb, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws, ws_bytes); break;
    case TDVP_OP_T: dispatch_b<T, TDVP_OP_T>(s, opb, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws, ws_bytes); break;
    case TDVP_OP_C: dispatch_b<T, TDVP_OP_C>(s, opb, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws, ws_bytes); break;
    case TDVP_OP_R: dispatch_b<T, TDVP_OP_R>(s, opb, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, ws, ws_bytes); break;
    default: TDVP_THROW(TDVP_ERR_ARG, "bad GEMM op_a");
  }
  HIP_CHECK(hipGetLastError());
}
template void gemm<double>(hipStream_t, int, int, int, int, int, zc, const void*, long long, long long,
                           const void*, long long, long long, zc, void*, long long, long long, int, void*, size_t);

template <typename T>
void gemm_heff(hipStream_t s, int M, int N, int K, const void* A, long long lda, const void* B, long long ldb,
               void* C, long long ldc, void* ws, size_t ws_bytes) {
  if (M <= 0 || N <= 0) return;
  launch_gemm<T, TDVP_OP_N, TDVP_OP_N, 1>(s, M, N, K, 1.0, A, lda, 0, B, ldb, 0, 0.0, C, ldc, 0, 1, ws, ws_bytes);
  HIP_CHECK(hipGetLastError());
}
template void gemm_heff<double>(hipStream_t, int, int, int, const void*, long long, const void*, long long, void*,
                                long long, void*, size_t);
template void gemm_heff<float>(hipStream_t, int, int, int, const void*, long long, const void*, long long, void*,
                               long long, void*, size_t);

template <typename T>
void gemm_heff_batched(hipStream_t s, int M, int N, int K, const void* A, long long lda, long long sa, const void* B,
                       long long ldb, long long sb, void* C, long long ldc, long long sc, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  launch_gemm<T, TDVP_OP_N, TDVP_OP_N, 1>(s, M, N, K, 1.0, A, lda, sa, B, ldb, sb, 0.0, C, ldc, sc, batch);
  HIP_CHECK(hipGetLastError());
}
template void gemm_heff_batched<double>(hipStream_t, int, int, int, const void*, long long, long long, const void*,
                                        long long, long long, void*, long long, long long, int);
template void gemm_heff_batched<float>(hipStream_t, int, int, int, const void*, long long, long long, const void*,
                                       long long, long long, void*, long long, long long, int);

template <typename T>
void gemm_nn_ws(hipStream_t s, int M, int N, int K, zc alpha, const void* A, long long lda, const void* B,
                long long ldb, zc beta, void* C, long long ldc, void* ws, size_t ws_bytes) {
  if (M <= 0 || N <= 0) return;
  launch_gemm<T, TDVP_OP_N, TDVP_OP_N, 0>(s, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1, ws,
                                          ws_bytes);
  HIP_CHECK(hipGetLastError());
}
template void gemm_nn_ws<double>(hipStream_t, int, int, int, zc, const void*, long long, const void*, long long, zc,
                                 void*, long long, void*, size_t);
template void gemm_nn_ws<float>(hipStream_t, int, int, int, zc, const void*, long long, const void*, long long, zc,
                                void*, long long, void*, size_t);
template void gemm<float>(hipStream_t, int, int, int, int, int, zc, const void*, long long, long long,
                          const void*, long long, long long, zc, void*, long long, long long, int, void*, size_t);

template <typename T>
void wapply(hipStream_t s, const WTable& t, const void* in, void* out, long long nP, long long nQ,
            long long isP, long long isQ, long long is1, long long is2, long long osP, long long osQ,
            long long os1, long long os2, const WCharges* wc) {
  if (nP <= 0 || nQ <= 0) return;
  if (nP > 65535) TDVP_THROW(TDVP_ERR_ARG, "wapply: P extent too large");
  dim3 grid((unsigned)((nQ + WQ - 1) / WQ), (unsigned)nP);
  const size_t sh = (size_t)t.n_in_ch * WQ * sizeof(typename VT<T>::c2);
  if (sh > 64 * 1024) TDVP_THROW(TDVP_ERR_ARG, "wapply: MPO bond dimension too large");
  WCharges w{nullptr, nullptr, nullptr, nullptr, 0};
  if (wc) {
    if (t.n_in_ch > WMAX_CH || t.n_out_ch > WMAX_CH) TDVP_THROW(TDVP_ERR_ARG, "wapply: too many charged channels");
    if (!wc->ql || !wc->qr || !wc->din || !wc->dout) TDVP_THROW(TDVP_ERR_ARG, "wapply: incomplete charge table");
    w = *wc;
  }
  hipLaunchKernelGGL(wapply_kernel<T>, grid, dim3(WNT), sh, s, static_cast<const T*>(in), static_cast<T*>(out),
                     nQ, isP, isQ, is1, is2, osP, osQ, os1, os2, t.rowptr, t.col,
                     reinterpret_cast<const double2*>(t.val), t.n_in_ch, t.n_out_ch, w);
  HIP_CHECK(hipGetLastError());
}
template void wapply<double>(hipStream_t, const WTable&, const void*, void*, long long, long long, long long,
                             long long, long long, long long, long long, long long, long long, long long,
                             const WCharges*);
template void wapply<float>(hipStream_t, const WTable&, const void*, void*, long long, long long, long long,
                            long long, long long, long long, long long, long long, long long, long long,
                            const WCharges*);

int zdots_blocks(long long n) { return (int)std::max<long long>(1, (n + DOT_CHUNK - 1) / DOT_CHUNK); }

void zdots(hipStream_t s, const void* V, long long ldv, int nv, const void* w, long long n, void* partial,
           int nb, void* out, bool conjugate) {
  if (nv <= 0) return;
  if (conjugate)
    hipLaunchKernelGGL(zdots_partial_kernel<true>, dim3(nb, nv), dim3(VNT), 0, s, static_cast<const double2*>(V), ldv,
                       nv, static_cast<const double2*>(w), n, static_cast<double2*>(partial));
  else
    hipLaunchKernelGGL(zdots_partial_kernel<false>, dim3(nb, nv), dim3(VNT), 0, s, static_cast<const double2*>(V), ldv,
                       nv, static_cast<const double2*>(w), n, static_cast<double2*>(partial));
  hipLaunchKernelGGL(zdots_final_kernel, dim3(nv), dim3(VNT), 0, s,
                     static_cast<const double2*>(partial), nb, nv, static_cast<double2*>(out));
  HIP_CHECK(hipGetLastError());
}

void zsum_partials(hipStream_t s, const void* partial, int nb, int nv, void* out) {
  if (nv <= 0) return;
  hipLaunchKernelGGL(zdots_final_kernel, dim3(nv), dim3(VNT), 0, s, static_cast<const double2*>(partial), nb, nv,
                     static_cast<double2*>(out));
  HIP_CHECK(hipGetLastError());
}

int zcombine_norm_blocks(long long n) { return (int)std::max<long long>(1, nblk(n, VNT)); }

void zdots_partial(hipStream_t s, const void* V, long long ldv, int nv, const void* w, long long n, void* partial,
                   int nb) {
  if (nv <= 0) return;
  hipLaunchKernelGGL(zdots_partial_kernel<true>, dim3(nb, nv), dim3(VNT), 0, s, static_cast<const double2*>(V), ldv,
                     nv, static_cast<const double2*>(w), n, static_cast<double2*>(partial));
  HIP_CHECK(hipGetLastError());
}

void zcombine_p(hipStream_t s, void* w, const void* V, long long ldv, int nv, const void* partial, int nb,
                double sign, long long n, void* cout, void* npart) {
  if (n <= 0 || nv <= 0) return;
  if (nv > ZC_MAXV) TDVP_THROW(TDVP_ERR_ARG, "zcombine_p: at most 64 vectors");
  if (npart)
    hipLaunchKernelGGL(zcombine_p_kernel<true>, dim3(nblk(n, VNT)), dim3(VNT), 0, s, static_cast<double2*>(w),
                       static_cast<const double2*>(V), ldv, nv, static_cast<const double2*>(partial), nb, sign, n,
                       static_cast<double2*>(cout), static_cast<double2*>(npart));
  else
    hipLaunchKernelGGL(zcombine_p_kernel<false>, dim3(nblk(n, VNT)), dim3(VNT), 0, s, static_cast<double2*>(w),
                       static_cast<const double2*>(V), ldv, nv, static_cast<const double2*>(partial), nb, sign, n,
                       static_cast<double2*>(cout), nullptr);
  HIP_CHECK(hipGetLastError());
}

void zcombine_dots(hipStream_t s, void* w, const void* V, long long ldv, int nv, const void* partial, int nb,
                   double sign, long long n, void* cout, void* dpart) {
  if (n <= 0 || nv <= 0) return;
  if (nv > ZC_MAXV) TDVP_THROW(TDVP_ERR_ARG, "zcombine_dots: at most 64 vectors");
  hipLaunchKernelGGL(zcombine_dots_kernel, dim3(nblk(n, VNT)), dim3(VNT), 0, s, static_cast<double2*>(w),
                     static_cast<const double2*>(V), ldv, nv, static_cast<const double2*>(partial), nb, sign, n,
                     static_cast<double2*>(cout), static_cast<double2*>(dpart));
  HIP_CHECK(hipGetLastError());
}

void zcombine(hipStream_t s, void* w, const void* V, long long ldv, int nv, const void* c, double sign,
              long long n) {
  if (n <= 0 || nv <= 0) return;
  hipLaunchKernelGGL(zcombine_kernel, dim3(nblk(n, VNT)), dim3(VNT), 0, s, static_cast<double2*>(w),
                     static_cast<const double2*>(V), ldv, nv, static_cast<const double2*>(c), sign, n);
  HIP_CHECK(hipGetLastError());
}

void zscale(hipStream_t s, void* dst, const void* src, zc a, long long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zscale_kernel, dim3(nblk(n)), dim3(256), 0, s, static_cast<double2*>(dst),
                     static_cast<const double2*>(src), a.real(), a.imag(), n);
  HIP_CHECK(hipGetLastError());
}

void zscale_invnorm(hipStream_t s, void* w, const void* partial, int np, void* out, long long n, void* host,
                    const void* coeffs, int ncoef, int host_norm_at) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zscale_invnorm_kernel, dim3(nblk(n, VNT)), dim3(VNT), 0, s, static_cast<double2*>(w),
                     static_cast<const double2*>(partial), np, static_cast<double2*>(out), n,
                     static_cast<double2*>(host), static_cast<const double2*>(coeffs), ncoef, host_norm_at);
  HIP_CHECK(hipGetLastError());
}

void z2c(hipStream_t s, void* dst, const void* src, long long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(z2c_kernel, dim3(nblk(n)), dim3(256), 0, s, static_cast<float2*>(dst),
                     static_cast<const double2*>(src), n);
  HIP_CHECK(hipGetLastError());
}

void c2z(hipStream_t s, void* dst, const void* src, long long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(c2z_kernel, dim3(nblk(n)), dim3(256), 0, s, static_cast<double2*>(dst),
                     static_cast<const float2*>(src), n);
  HIP_CHECK(hipGetLastError());
}

void copy2d(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
            long long cols, int esize) {
  if (rows <= 0 || cols <= 0) return;
  if (esize == 16)
    hipLaunchKernelGGL(copy2d_kernel<double2>, dim3(nblk(rows * cols)), dim3(256), 0, s, static_cast<double2*>(dst),
                       ldd, static_cast<const double2*>(src), lds, rows, cols);
  else
    hipLaunchKernelGGL(copy2d_kernel<float2>, dim3(nblk(rows * cols)), dim3(256), 0, s, static_cast<float2*>(dst),
                       ldd, static_cast<const float2*>(src), lds, rows, cols);
  HIP_CHECK(hipGetLastError());
}

void ztri(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
          long long cols, int mode) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(ztri_kernel, dim3(nblk(rows * cols)), dim3(256), 0, s, static_cast<double2*>(dst), ldd,
                     static_cast<const double2*>(src), lds, rows, cols, mode);
  HIP_CHECK(hipGetLastError());
}

void zconjtrans(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
                long long cols) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(zconjtrans_kernel, dim3(nblk(rows * cols)), dim3(256), 0, s, static_cast<double2*>(dst),
                     ldd, static_cast<const double2*>(src), lds, rows, cols);
  HIP_CHECK(hipGetLastError());
}

void zhermitize(hipStream_t s, void* A, long long n) { zhermitize_to(s, A, A, n); }

void zhermitize_to(hipStream_t s, void* A, const void* S, long long n, int* zero, int nzero) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zhermitize_kernel, dim3(nblk(n * n)), dim3(256), 0, s, static_cast<double2*>(A),
                     static_cast<const double2*>(S), n, zero, nzero);
  HIP_CHECK(hipGetLastError());
}

void zfill(hipStream_t s, void* dst, zc v, long long n, int esize) {
  if (n <= 0) return;
  if (esize == 16)
    hipLaunchKernelGGL(fill_kernel<double2>, dim3(nblk(n)), dim3(256), 0, s, static_cast<double2*>(dst),
                       make_double2(v.real(), v.imag()), n);
  else
    hipLaunchKernelGGL(fill_kernel<float2>, dim3(nblk(n)), dim3(256), 0, s, static_cast<float2*>(dst),
                       make_float2(float(v.real()), float(v.imag())), n);
  HIP_CHECK(hipGetLastError());
}

template <bool PACK>
void rows_pack_dispatch(hipStream_t s, void* packed, int pe, void* dense, int de, int rows, long long ld, const int* seg,
                        int maxlen) {
  if (rows <= 0 || maxlen <= 0) return;
  if (rows > 65535) TDVP_THROW(TDVP_ERR_ARG, "row segments: too many rows");
  const dim3 grid((unsigned)((maxlen + 255) / 256), (unsigned)rows);
  if (pe == 16 && de == 16)
    hipLaunchKernelGGL((rows_pack_kernel<double2, double2, PACK>), grid, dim3(256), 0, s, static_cast<double2*>(packed),
                       static_cast<double2*>(dense), rows, ld, seg);
  else if (pe == 16 && de == 8)
    hipLaunchKernelGGL((rows_pack_kernel<double2, float2, PACK>), grid, dim3(256), 0, s, static_cast<double2*>(packed),
                       static_cast<float2*>(dense), rows, ld, seg);
  else
    TDVP_THROW(TDVP_ERR_ARG, "row segments: unsupported element sizes");
  HIP_CHECK(hipGetLastError());
}
void pack_rows(hipStream_t s, void* packed, int packed_esize, const void* dense, int dense_esize, int rows, long long ld,
               const int* seg, int maxlen) {
  rows_pack_dispatch<true>(s, packed, packed_esize, const_cast<void*>(dense), dense_esize, rows, ld, seg, maxlen);
}
void unpack_rows(hipStream_t s, void* dense, int dense_esize, const void* packed, int packed_esize, int rows,
                 long long ld, const int* seg, int maxlen) {
  rows_pack_dispatch<false>(s, const_cast<void*>(packed), packed_esize, dense, dense_esize, rows, ld, seg, maxlen);
}

void zrandom_blocks(hipStream_t s, void* E, int R, int C, const int* qr, const int* qc, unsigned long long seed) {
  const long long n = (long long)R * C;
  if (n <= 0) return;
  hipLaunchKernelGGL(zrandom_blocks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, static_cast<double2*>(E),
                     R, C, qr, qc, seed);
  HIP_CHECK(hipGetLastError());
}

void zscale_phys(hipStream_t s, void* G, long long nx, long long nq, double f0, double f1) {
  if (nx <= 0 || nq <= 0) return;
  hipLaunchKernelGGL(zscale_phys_kernel, dim3(nblk(nx * 2 * nq)), dim3(256), 0, s, static_cast<double2*>(G),
                     nx, nq, f0, f1);
  HIP_CHECK(hipGetLastError());
}

void zshift_diag(hipStream_t s, void* G, long long n, double a, double b) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zshift_diag_kernel, dim3(nblk(n * n)), dim3(256), 0, s, static_cast<double2*>(G), n, a, b);
  HIP_CHECK(hipGetLastError());
}

void zscale_rows(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
                 long long cols, const double* f) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(zscale_rc_kernel, dim3(nblk(rows * cols)), dim3(256), 0, s, static_cast<double2*>(dst), ldd,
                     static_cast<const double2*>(src), lds, rows, cols, f, 0);
  HIP_CHECK(hipGetLastError());
}

void zscale_cols(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
                 long long cols, const double* f) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(zscale_rc_kernel, dim3(nblk(rows * cols)), dim3(256), 0, s, static_cast<double2*>(dst), ldd,
                     static_cast<const double2*>(src), lds, rows, cols, f, 1);
  HIP_CHECK(hipGetLastError());
}

void zgather(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, const int* ridx, long long nr,
             const int* cidx, long long nc) {
  if (nr <= 0 || nc <= 0) return;
  hipLaunchKernelGGL(zgather_kernel, dim3(nblk(nr * nc)), dim3(256), 0, s, static_cast<double2*>(dst), ldd,
                     static_cast<const double2*>(src), lds, ridx, nr, cidx, nc);
  HIP_CHECK(hipGetLastError());
}

void zscatter(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, const int* ridx, long long nr,
              const int* cidx, long long nc) {
  if (nr <= 0 || nc <= 0) return;
  hipLaunchKernelGGL(zscatter_kernel, dim3(nblk(nr * nc)), dim3(256), 0, s, static_cast<double2*>(dst), ldd,
                     static_cast<const double2*>(src), lds, ridx, nr, cidx, nc);
  HIP_CHECK(hipGetLastError());
}

void zscatter_cols(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long nr,
                   const int* cidx, long long nc) {
  zscatter(s, dst, ldd, src, lds, nullptr, nr, cidx, nc);
}

void zunit_blocks(hipStream_t s, void* diag, const void* H, long long n, const int* idx, const int* pos, int cnt,
                  void* rows) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(zunit_blocks_kernel, dim3(nblk(cnt)), dim3(256), 0, s, static_cast<double2*>(diag),
                     static_cast<const double2*>(H), n, idx, pos, cnt, static_cast<double2*>(rows));
  HIP_CHECK(hipGetLastError());
}

}  // namespace kern
