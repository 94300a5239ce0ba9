// Tall-skinny block kernels: Gram products X^T Y with FP64 accumulation (deterministic two-stage
// reduction; FP32 accumulation within row chunks on request for nearly orthonormal FP32 blocks), block
// rotations X V, residual norms, conversions and the random start block.
#include <algorithm>
#include <cmath>
#include <vector>

#include "rw_internal.h"

namespace rw {

// ---------------------------------------------------------------------------------------------
// Gram: G = X^T Y.  Stage 1: block (tx, ty, chunk) computes a 64 x 64 tile of the product over a
// chunk of rows, staging 32-row slabs of X and Y in LDS as FP64; each of the 256 threads owns a
// 4 x 4 sub-tile (rows tx + 16 a, cols ty + 16 b).  Stage 2 sums the chunk partials in order.
// FP32 x FP32 products are exact in FP64, so FP32 inputs lose nothing before the accumulation.
// ---------------------------------------------------------------------------------------------
constexpr int kGT = 64;      // tile edge
constexpr int kGK = 32;      // rows per LDS slab
constexpr int64_t kGramRowsPerChunk = 4096;

static int64_t gram_chunks(int64_t rows, int bx, int by) {
  int64_t tiles = (int64_t)((bx + kGT - 1) / kGT) * ((by + kGT - 1) / kGT);
  int64_t want = std::max<int64_t>(1, 2048 / std::max<int64_t>(1, tiles));
  int64_t by_rows = (rows + kGramRowsPerChunk - 1) / kGramRowsPerChunk;
  int64_t c = std::min<int64_t>(want, by_rows);
  return std::max<int64_t>(1, c);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gram(const T* X, int64_t ldx, const T* Y, int64_t ldy,
                                              int64_t rows, int bx, int by, int64_t chunk_rows,
                                              double* out, int64_t out_stride) {
  __shared__ double sX[kGK][kGT + 1];
  __shared__ double sY[kGK][kGT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.x * kGT, j0 = blockIdx.y * kGT;
  const int64_t r_begin = blockIdx.z * chunk_rows;
  const int64_t r_end = std::min<int64_t>(rows, r_begin + chunk_rows);
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const int lr = threadIdx.x & 31;      // row within slab
  const int lc = threadIdx.x >> 5;      // 0..7: column group
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGK) {
    const int64_t row = r0 + lr;
    const bool rin = row < r_end;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int col = lc + 8 * k;
      int ci = i0 + col, cj = j0 + col;
      sX[lr][col] = (rin && ci < bx) ? (double)Elem<T>::ld(X, (int64_t)ci * ldx + row) : 0.0;
      sY[lr][col] = (rin && cj < by) ? (double)Elem<T>::ld(Y, (int64_t)cj * ldy + row) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kGK; ++k) {
      double xv[4], yv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xv[a] = sX[k][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) yv[b] = sY[k][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xv[a], yv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* o = out + blockIdx.z * out_stride;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
      if (i < bx && j < by) o[(int64_t)j * bx + i] = acc[a][b];
    }
}

// Large Gram products on the FP64 matrix cores (v_mfma_f64_16x16x4f64: A(i,k) from lane i + 16k,
// B(k,j) from lane j + 16k, D(4v + l/16, l%16) in register v of lane l).  One wave computes a 32 x 32 tile
// of X^T Y over a chunk of rows.  The contraction order inside a 32-row step is free, so lane l takes
// rows r0 + 8 (l/16) + s for MFMA step s: each lane reads 8 consecutive rows of its column, and the four
// 16-lane groups together read 32 consecutive rows (whole cache lines).  Inputs are widened to FP64 in
// registers (FP32 x FP32 products are exact in FP64).  With `sym` (X^T Y known to be symmetric) only
// tiles on or above the diagonal are computed and off-diagonal ones are written to both places; a
// diagonal tile of X^T X loads its operand once.
typedef double gram_d4 __attribute__((ext_vector_type(4)));
constexpr int kGM = 32;        // tile edge
constexpr int kGMRows = 32;    // rows per step (8 MFMA steps)

// 8 consecutive rows of one column; vector loads when the run is whole and aligned (vec: the leading
// dimension is a multiple of 8 elements and the base 32-byte aligned, so col + r is aligned for r = 0 mod 8)
template <typename T>
__device__ __forceinline__ void gram_load8(const T* col, int64_t r, int64_t r_end, bool ok, bool vec, T (&v)[8]) {
  if (ok && vec && r + 8 <= r_end) {
    const uint4* p = reinterpret_cast<const uint4*>(col + r);
    constexpr int nq = (int)(8 * sizeof(T) / sizeof(uint4));
    uint4 q[nq];
#pragma unroll
    for (int i = 0; i < nq; ++i) q[i] = p[i];
    __builtin_memcpy(v, q, sizeof(q));
  } else {
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = (ok && r + s < r_end) ? col[r + s] : T(0);
  }
}

// SPLIT waves per workgroup: wave w takes the w-th of SPLIT row ranges of the chunk, and the waves' tiles
// are added in wave order through LDS (short reductions: fewer sequential steps per wave)
template <typename T, int SPLIT>
__global__ __launch_bounds__(64 * SPLIT) void k_gram_mfma(const T* X, int64_t ldx, const T* Y, int64_t ldy,
                                                          int64_t rows, int bx, int by, int64_t chunk_rows,
                                                          int tiles_x, int sym, int vec, double* out,
                                                          int64_t out_stride) {
  int ti, tj;
  const int t = blockIdx.x;
  if (sym) {   // upper triangle of tiles, column by column
    tj = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((tj + 1) * (tj + 2) / 2 <= t) ++tj;
    while (tj * (tj + 1) / 2 > t) --tj;
    ti = t - tj * (tj + 1) / 2;
  } else {
    ti = t % tiles_x;
    tj = t / tiles_x;
  }
  const int i0 = ti * kGM, j0 = tj * kGM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c16 = lane & 15, kq = lane >> 4;
  const int64_t sub_rows = (chunk_rows / SPLIT + kGMRows - 1) / kGMRows * kGMRows;
  const int64_t c_begin = (int64_t)blockIdx.y * chunk_rows;
  const int64_t c_end = std::min<int64_t>(rows, c_begin + chunk_rows);
  const int64_t r_begin = std::min<int64_t>(c_end, c_begin + wave * sub_rows);
  const int64_t r_end = wave == SPLIT - 1 ? c_end : std::min<int64_t>(c_end, r_begin + sub_rows);
  const bool same = ti == tj && X == Y && ldx == ldy && i0 == j0;   // B operand equals A operand
  const int ca0 = i0 + c16, ca1 = i0 + 16 + c16, cb0 = j0 + c16, cb1 = j0 + 16 + c16;
  const bool oa0 = ca0 < bx, oa1 = ca1 < bx, ob0 = cb0 < by, ob1 = cb1 < by;
  const T* pa0 = X + (int64_t)(oa0 ? ca0 : 0) * ldx;
  const T* pa1 = X + (int64_t)(oa1 ? ca1 : 0) * ldx;
  const T* pb0 = Y + (int64_t)(ob0 ? cb0 : 0) * ldy;
  const T* pb1 = Y + (int64_t)(ob1 ? cb1 : 0) * ldy;
  gram_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = gram_d4{0.0, 0.0, 0.0, 0.0};
  // raw values of the next two steps (widened when used): loads run two steps ahead of the MFMAs
  T q[2][4][8];
  auto fetch = [&](int64_t r0, T (&d)[4][8]) {
    const int64_t r = r0 + 8 * kq;
    gram_load8(pa0, r, r_end, oa0, vec, d[0]);
    gram_load8(pa1, r, r_end, oa1, vec, d[1]);
    if (!same) {
      gram_load8(pb0, r, r_end, ob0, vec, d[2]);
      gram_load8(pb1, r, r_end, ob1, vec, d[3]);
    }
  };
  if (r_begin < r_end) fetch(r_begin, q[0]);
  if (r_begin + kGMRows < r_end) fetch(r_begin + kGMRows, q[1]);
  for (int64_t r00 = r_begin; r00 < r_end; r00 += 2 * kGMRows) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r0 = r00 + h * kGMRows;
      if (r0 >= r_end) break;
      T cur[4][8];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = 0; e < 8; ++e) cur[c][e] = (same && c >= 2) ? q[h][c - 2][e] : q[h][c][e];
      if (r0 + 2 * kGMRows < r_end) fetch(r0 + 2 * kGMRows, q[h]);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double xa[2] = {(double)Elem<T>::ld(cur[0], e), (double)Elem<T>::ld(cur[1], e)};
        const double xb[2] = {(double)Elem<T>::ld(cur[2], e), (double)Elem<T>::ld(cur[3], e)};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a], xb[b], acc[a][b], 0, 0, 0);
      }
    }
  }
  if (SPLIT > 1) {
    __shared__ double red[SPLIT > 1 ? SPLIT - 1 : 1][16][64];
    if (wave > 0) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) red[wave - 1][(a * 2 + b) * 4 + v][lane] = acc[a][b][v];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 1; w < SPLIT; ++w)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[a][b][v] += red[w - 1][(a * 2 + b) * 4 + v][lane];
  }
  double* o = out + (int64_t)blockIdx.y * out_stride;
  const bool mirror = sym && ti != tj;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 16 * a + 4 * v + kq, j = j0 + 16 * b + c16;
        if (i < bx && j < by) {
          o[(int64_t)j * bx + i] = acc[a][b][v];
          if (mirror) o[(int64_t)i * bx + j] = acc[a][b][v];
        }
      }
}

// ---------------------------------------------------------------------------------------------
// Symmetric Gram of tall FP32 blocks, G = X^T Y where X^T Y is symmetric (Y = X, or Y = op X for a
// symmetric op), on the FP32 matrix cores.  One workgroup per chunk of rows: 32-row slabs of X and Y pass
// through LDS (column-major with a 36-float column stride, double-buffered; the next slab waits in
// registers while the current one is used), and the 16 waves share the 16 x 16 blocks of the upper block
// triangle, grouped in 32 x 32 tiles whose fragments serve two blocks each.  Row 8 g + e of the slab is
// the k index g of MFMA step e (A(i,k) and B(k,j) from lane i + 16 k or j + 16 k, D(4 (l/16) + v, l%16)
// in register v of lane l).  A chunk (at most 2048 rows) accumulates in FP32, so its rounding error
// stays near FP32's unit roundoff relative to the column norms; the chunk partials (FP32, upper
// entries) are summed over chunks in FP64 and in chunk order.
// ---------------------------------------------------------------------------------------------
constexpr int kSGRows = 32;
constexpr int kSGStride = 36;     // b128 reads of 8 lanes in one column group fall in distinct banks
constexpr int kSGMaxN = 224;      // 7 tiles of 32
constexpr int kSGWaves = 16;
constexpr int kSGMaxTiles = 2;
constexpr int kSGSlab = kSGMaxN * kSGStride;   // floats per matrix slab in LDS

struct SymGramPlan {
  unsigned char tile[28];              // (tj << 3) | ti, ti <= tj; wave w owns tile[first[w] .. first[w + 1])
  unsigned char first[kSGWaves + 1];
};

typedef float sg_f4 __attribute__((ext_vector_type(4)));

template <bool SAME>
__global__ __launch_bounds__(64 * kSGWaves) void k_gram_sym_f32(const float* X, const float* Y, int64_t ld,
                                                                int64_t rows, int nb, int64_t chunk_rows, int vec,
                                                                SymGramPlan plan, float* partial) {
  constexpr int NM = SAME ? 1 : 2;
  extern __shared__ float sg[];   // [2 buffers][NM][kSGSlab]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, c16 = lane & 15, g = lane >> 4;
  const int64_t r_begin = (int64_t)blockIdx.x * chunk_rows;
  const int64_t r_end = std::min<int64_t>(rows, r_begin + chunk_rows);
  const int nslab = (int)((r_end - r_begin + kSGRows - 1) / kSGRows);
  const int nq = ((nb + 15) & ~15) * (kSGRows / 4);   // float4 per matrix slab (columns padded to 16)
  float4 pre[2][NM];
  auto fetch = [&](int s) {
    const int64_t r0 = r_begin + (int64_t)s * kSGRows;
    const bool full = vec && r0 + kSGRows <= r_end;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = tid + 64 * kSGWaves * u;
      const int col = q >> 3;
      const int64_t row = r0 + 4 * (q & 7);
#pragma unroll
      for (int mt = 0; mt < NM; ++mt) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (q < nq && col < nb) {
          const float* p = (mt == 0 ? X : Y) + (int64_t)col * ld + row;
          if (full) {
            v = *reinterpret_cast<const float4*>(p);
          } else {
            if (row + 0 < r_end) v.x = p[0];
            if (row + 1 < r_end) v.y = p[1];
            if (row + 2 < r_end) v.z = p[2];
            if (row + 3 < r_end) v.w = p[3];
          }
        }
        pre[u][mt] = v;
      }
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = tid + 64 * kSGWaves * u;
      if (q < nq) {
#pragma unroll
        for (int mt = 0; mt < NM; ++mt)
          *reinterpret_cast<float4*>(sg + (b * NM + mt) * kSGSlab + (q >> 3) * kSGStride + 4 * (q & 7)) = pre[u][mt];
      }
    }
  };
  const int t_first = plan.first[wave], cnt = plan.first[wave + 1] - t_first;
  sg_f4 acc[kSGMaxTiles][2][2];
#pragma unroll
  for (int t = 0; t < kSGMaxTiles; ++t)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[t][a][b] = sg_f4{0.f, 0.f, 0.f, 0.f};
  if (nslab > 0) {
    fetch(0);
    stash(0);
    if (nslab > 1) fetch(1);
  }
  __syncthreads();
  for (int s = 0; s < nslab; ++s) {
    const float* sx = sg + (s & 1) * NM * kSGSlab;
    const float* sy = SAME ? sx : sx + kSGSlab;
#pragma unroll
    for (int t = 0; t < kSGMaxTiles; ++t) {
      if (t >= cnt) break;
      const int code = plan.tile[t_first + t], ti = code & 7, tj = code >> 3;
      const bool a1 = 32 * ti + 16 < nb, b1 = 32 * tj + 16 < nb, diag = ti == tj;
      float fa[2][8], fb[2][8];
      auto frag = [&](const float* base, int col, float (&f)[8]) {
        const float4 lo = *reinterpret_cast<const float4*>(base + col * kSGStride + 8 * g);
        const float4 hi = *reinterpret_cast<const float4*>(base + col * kSGStride + 8 * g + 4);
        f[0] = lo.x; f[1] = lo.y; f[2] = lo.z; f[3] = lo.w;
        f[4] = hi.x; f[5] = hi.y; f[6] = hi.z; f[7] = hi.w;
      };
      frag(sx, 32 * ti + c16, fa[0]);
      frag(sx, 32 * ti + 16 + c16, fa[1]);   // beyond nb only when !a1: read but unused (inside the slab)
      if (SAME && diag) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          fb[0][e] = fa[0][e];
          fb[1][e] = fa[1][e];
        }
      } else {
        frag(sy, 32 * tj + c16, fb[0]);
        frag(sy, 32 * tj + 16 + c16, fb[1]);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        acc[t][0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0][e], fb[0][e], acc[t][0][0], 0, 0, 0);
        if (b1) acc[t][0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0][e], fb[1][e], acc[t][0][1], 0, 0, 0);
        if (a1 && !diag) acc[t][1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[1][e], fb[0][e], acc[t][1][0], 0, 0, 0);
        if (a1 && b1) acc[t][1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[1][e], fb[1][e], acc[t][1][1], 0, 0, 0);
      }
    }
    if (s + 1 < nslab) stash((s + 1) & 1);
    __syncthreads();
    if (s + 2 < nslab) fetch(s + 2);
  }
  float* o = partial + (int64_t)blockIdx.x * nb * nb;   // o[i nb + j], i <= j (16-block upper triangle)
#pragma unroll
  for (int t = 0; t < kSGMaxTiles; ++t) {
    if (t >= cnt) break;
    const int code = plan.tile[t_first + t], ti = code & 7, tj = code >> 3;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (ti == tj && a == 1 && b == 0) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 32 * ti + 16 * a + 4 * g + v, j = 32 * tj + 16 * b + c16;
          if (i < nb && j < nb) o[(int64_t)i * nb + j] = acc[t][a][b][v];
        }
      }
  }
}

// G (nb x nb, symmetric) = sum over chunks of the upper entries in FP64: a block covers 64 consecutive
// entries, its four waves take every fourth chunk, and the four sums are added in wave order
__global__ __launch_bounds__(256) void k_sum_sym_f32(const float* partial, int64_t nch, int nb, double* G) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t k = blockIdx.x * (int64_t)64 + lane;
  const int64_t nn = (int64_t)nb * nb;
  double s = 0.0;
  if (k < nn) {
#pragma unroll 4
    for (int64_t c = wave; c < nch; c += 4) s += (double)partial[c * nn + k];
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && k < nn) {
    const int i = (int)(k / nb), j = (int)(k % nb);
    if (i <= j) {
      const double t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
      G[(int64_t)j * nb + i] = t;
      G[(int64_t)i * nb + j] = t;
    }
  }
}

// chunks: one per CU at least 512 rows each, at most 2048 rows each
static int64_t sym_gram_chunks(int64_t rows) {
  const int64_t a = std::min<int64_t>(256, (rows + 511) / 512), b = (rows + 2047) / 2048;
  return std::max<int64_t>(1, std::max(a, b));
}

static bool sym_gram_fits(int64_t rows, int nb) { return nb >= 96 && nb <= kSGMaxN && rows >= 4096; }

// tiles of the upper triangle to waves: largest first, each to the wave whose SIMD (wave % 4) and then
// itself carry the least work (a tile's work is its number of 16 x 16 blocks)
static bool sym_gram_plan(int nb, SymGramPlan* p) {
  const int T = (nb + 31) / 32;
  struct Tl { int code, cost; };
  std::vector<Tl> tl;
  for (int tj = 0; tj < T; ++tj)
    for (int ti = 0; ti <= tj; ++ti) {
      const int na = 32 * ti + 16 < nb ? 2 : 1, nbk = 32 * tj + 16 < nb ? 2 : 1;
      int cost = na * nbk;
      if (ti == tj && na == 2) cost -= 1;
      tl.push_back({(tj << 3) | ti, cost});
    }
  std::stable_sort(tl.begin(), tl.end(), [](const Tl& x, const Tl& y) { return x.cost > y.cost; });
  int load[kSGWaves] = {0}, simd[4] = {0};
  std::vector<int> own[kSGWaves];
  for (const Tl& t : tl) {
    int best = 0;
    for (int w = 1; w < kSGWaves; ++w) {
      const int sw = simd[w & 3], sb = simd[best & 3];
      if (sw < sb || (sw == sb && load[w] < load[best])) best = w;
    }
    own[best].push_back(t.code);
    load[best] += t.cost;
    simd[best & 3] += t.cost;
  }
  int pos = 0;
  for (int w = 0; w < kSGWaves; ++w) {
    if ((int)own[w].size() > kSGMaxTiles) return false;
    p->first[w] = (unsigned char)pos;
    for (int c : own[w]) p->tile[pos++] = (unsigned char)c;
  }
  p->first[kSGWaves] = (unsigned char)pos;
  return true;
}

static bool gram_sym_f32(const float* X, int64_t ldx, const float* Y, int64_t ldy, int64_t rows, int nb, double* G,
                         double* partial, hipStream_t s) {
  if (ldx != ldy || !sym_gram_fits(rows, nb)) return false;
  SymGramPlan plan;
  if (!sym_gram_plan(nb, &plan)) return false;
  const int64_t nch = sym_gram_chunks(rows);
  const int64_t chunk_rows = ((rows + nch - 1) / nch + kSGRows - 1) / kSGRows * kSGRows;
  const int64_t nblk = (rows + chunk_rows - 1) / chunk_rows;
  const bool same = X == Y;
  const int vec = (ldx % 4 == 0 && (uintptr_t)X % 16 == 0 && (uintptr_t)Y % 16 == 0) ? 1 : 0;
  const size_t sh = (size_t)2 * (same ? 1 : 2) * kSGSlab * sizeof(float);
  float* part = reinterpret_cast<float*>(partial);
  if (same) {
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_gram_sym_f32<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
      attr = true;
    }
    k_gram_sym_f32<true><<<(unsigned)nblk, 64 * kSGWaves, sh, s>>>(X, Y, ldx, rows, nb, chunk_rows, vec, plan, part);
  } else {
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_gram_sym_f32<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
      attr = true;
    }
    k_gram_sym_f32<false><<<(unsigned)nblk, 64 * kSGWaves, sh, s>>>(X, Y, ldx, rows, nb, chunk_rows, vec, plan, part);
  }
  k_sum_sym_f32<<<(unsigned)(((int64_t)nb * nb + 63) / 64), 256, 0, s>>>(part, nblk, nb, G);
  return true;
}

__global__ void k_sum_chunks(const double* partial, int64_t count, int64_t nchunks, double* G) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= count) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunks; ++c) s += partial[c * count + k];
  G[k] = s;
}

// ---------------------------------------------------------------------------------------------
// Projection P = Q^T X of a tall basis (N x m, column-major) on a few label maps (X: C x N, label-major):
// blocks over (2048-row chunk, 8 columns); each thread holds its 8 rows of up to 4 labels of X in registers
// and accumulates the 8 x 4 products in FP64 (products of FP32 values are exact), then one DPP wave sum per
// (column, label) and the four waves in order.  Q is read once; X once per 8 columns (from cache).  The chunk
// partials are summed in a fixed order.
// ---------------------------------------------------------------------------------------------
constexpr int kPcRowsPerThread = 8;
constexpr int kPcRows = 256 * kPcRowsPerThread;
constexpr int kPcCols = 8;
constexpr int kPcLabels = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_project_cols(const T* Q, int64_t N, int m, const T* X, int C, int l0,
                                                      double* partial) {
  __shared__ double sh[4][kPcCols * kPcLabels];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t chunk = blockIdx.x;
  const int j0 = (int)blockIdx.y * kPcCols;
  const int ncol = min(kPcCols, m - j0), nl = min(kPcLabels, C - l0);
  int64_t ic[kPcRowsPerThread];
  double x[kPcRowsPerThread][kPcLabels];
#pragma unroll
  for (int q = 0; q < kPcRowsPerThread; ++q) {
    const int64_t i = chunk * kPcRows + tid + 256 * q;
    ic[q] = i < N ? i : N - 1;
#pragma unroll
    for (int k = 0; k < kPcLabels; ++k)
      x[q][k] = (i < N && k < nl) ? (double)X[(int64_t)(l0 + k) * N + i] : 0.0;
  }
  double acc[kPcCols][kPcLabels];
#pragma unroll
  for (int jj = 0; jj < kPcCols; ++jj) {
    const T* qc = Q + (int64_t)(j0 + min(jj, ncol - 1)) * N;
    double v[kPcRowsPerThread];
#pragma unroll
    for (int q = 0; q < kPcRowsPerThread; ++q) v[q] = (double)qc[ic[q]];
#pragma unroll
    for (int k = 0; k < kPcLabels; ++k) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < kPcRowsPerThread; ++q) a += v[q] * x[q][k];
      acc[jj][k] = a;
    }
  }
#pragma unroll
  for (int jj = 0; jj < kPcCols; ++jj)
#pragma unroll
    for (int k = 0; k < kPcLabels; ++k) {
      const double t = wave_sum64(acc[jj][k]);
      if (lane == 0) sh[wave][jj * kPcLabels + k] = t;
    }
  __syncthreads();
  if (tid < kPcCols * kPcLabels) {
    const int jj = tid / kPcLabels, k = tid % kPcLabels;
    if (jj < ncol && k < nl) {
      const double t = (sh[0][tid] + sh[1][tid]) + (sh[2][tid] + sh[3][tid]);
      partial[chunk * ((int64_t)m * C) + (j0 + jj) + (int64_t)(l0 + k) * m] = t;
    }
  }
}

size_t project_cols_partial_count(int64_t N, int m, int C) {
  return (size_t)((N + kPcRows - 1) / kPcRows) * m * C;
}

int project_cols(int dt, const void* Q, int64_t N, int m, const void* X, int C, double* P, double* partial,
                 hipStream_t s) {
  if (m <= 0 || C <= 0) return RW_OK;
  const int64_t nch = (N + kPcRows - 1) / kPcRows;
  const dim3 grid((unsigned)nch, (unsigned)((m + kPcCols - 1) / kPcCols));
  for (int l0 = 0; l0 < C; l0 += kPcLabels) {
    if (dt == RW_F64)
      k_project_cols<double><<<grid, 256, 0, s>>>((const double*)Q, N, m, (const double*)X, C, l0, partial);
    else
      k_project_cols<float><<<grid, 256, 0, s>>>((const float*)Q, N, m, (const float*)X, C, l0, partial);
    RW_LAUNCH_CHECK();
  }
  k_sum_chunks<<<nblocks((int64_t)m * C, 256), 256, 0, s>>>(partial, (int64_t)m * C, nch, P);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

static int gram_mfma_tiles(int bx, int by, bool sym) {
  const int tx = (bx + kGM - 1) / kGM, ty = (by + kGM - 1) / kGM;
  return sym ? tx * (tx + 1) / 2 : tx * ty;
}

static int64_t gram_big_chunks(int64_t rows, int bx, int by, bool sym) {
  // about 4096 waves (four per SIMD), at least 256 rows per chunk
  const int64_t tiles = gram_mfma_tiles(bx, by, sym);
  const int64_t want = std::max<int64_t>(1, 4096 / std::max<int64_t>(1, tiles));
  const int64_t by_rows = std::max<int64_t>(1, rows / 256);
  return std::max<int64_t>(1, std::min<int64_t>(want, by_rows));
}

// the matrix-core kernel for wide products, and for short ones (the small dense systems: at most 4096 rows)
// from 32 columns on, where the VALU kernel's 64 x 64 tiles leave most of the chip idle
static bool gram_is_big(int64_t rows, int bx, int by) {
  return (bx >= 96 && by >= 96) || (rows <= 4096 && bx >= 32 && by >= 32);
}

size_t gram_partial_count(int64_t rows, int bx, int by) {
  // the symmetric case has the most chunks (fewer tiles)
  int64_t nch = gram_is_big(rows, bx, by) ? gram_big_chunks(rows, bx, by, bx == by) : gram_chunks(rows, bx, by);
  size_t c = (size_t)nch * bx * by;
  // FP32 partials of the symmetric FP32 kernel, for any width up to bx (callers may use fewer columns)
  const int sb = std::min(bx, kSGMaxN);
  if (bx == by && sym_gram_fits(rows, sb)) c = std::max(c, ((size_t)sym_gram_chunks(rows) * sb * sb + 1) / 2);
  return c;
}

// FP64 Gram with few columns of Y over a short range of rows: one wave per column of X, lanes stride the
// rows, a butterfly per product (fixed order)
__global__ __launch_bounds__(64) void k_gram_skinny(const double* X, int64_t ldx, const double* Y, int64_t ldy,
                                                     int64_t rows, int bx, int by, double* G) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const double* xi = X + (int64_t)i * ldx;
  for (int j = 0; j < by; ++j) {
    const double* yj = Y + (int64_t)j * ldy;
    double acc = 0.0;
    for (int64_t r = lane; r < rows; r += 64) acc += xi[r] * yj[r];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) G[(int64_t)j * bx + i] = acc;
  }
}

int gram(int dt, const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t rows, int bx, int by,
         double* G, double* partial, hipStream_t s, bool sym, bool acc32) {
  if (bx <= 0 || by <= 0) return RW_OK;
  if (dt == RW_F64 && by <= 8 && bx > by && rows <= 8192) {
    k_gram_skinny<<<bx, 64, 0, s>>>((const double*)X, ldx, (const double*)Y, ldy, rows, bx, by, G);
    RW_LAUNCH_CHECK();
    return RW_OK;
  }
  if (acc32 && dt == RW_F32 && sym && bx == by &&
      gram_sym_f32((const float*)X, ldx, (const float*)Y, ldy, rows, bx, G, partial, s)) {
    RW_LAUNCH_CHECK();
    return RW_OK;
  }
  const bool big = gram_is_big(rows, bx, by);
  const int slab = big ? kGMRows : kGK;
  const int sy = (sym && bx == by) ? 1 : 0;
  int64_t nch = big ? gram_big_chunks(rows, bx, by, sy != 0) : gram_chunks(rows, bx, by);
  int64_t chunk_rows = (rows + nch - 1) / nch;
  chunk_rows = (chunk_rows + slab - 1) / slab * slab;
  if (chunk_rows == 0) chunk_rows = slab;
  nch = std::max<int64_t>(1, (rows + chunk_rows - 1) / chunk_rows);
  int64_t count = (int64_t)bx * by;
  double* dst = nch == 1 ? G : partial;
  if (big) {
    const int tiles_x = (bx + kGM - 1) / kGM;
    dim3 grid((unsigned)gram_mfma_tiles(bx, by, sy != 0), (unsigned)nch);
    const size_t es = dtype_size(dt);
    const int vec = (ldx % 8 == 0 && ldy % 8 == 0 && (uintptr_t)X % (8 * es) == 0 && (uintptr_t)Y % (8 * es) == 0) ? 1 : 0;
    if (nch == 1 && rows <= 4096) {   // short products (the small dense matrices): four waves per tile
      if (dt == RW_F64)
        k_gram_mfma<double, 4><<<grid, 256, 0, s>>>((const double*)X, ldx, (const double*)Y, ldy, rows, bx, by, chunk_rows, tiles_x, sy, vec, dst, count);
      else if (dt == RW_F32)
        k_gram_mfma<float, 4><<<grid, 256, 0, s>>>((const float*)X, ldx, (const float*)Y, ldy, rows, bx, by, chunk_rows, tiles_x, sy, vec, dst, count);
      else
        k_gram_mfma<uint16_t, 4><<<grid, 256, 0, s>>>((const uint16_t*)X, ldx, (const uint16_t*)Y, ldy, rows, bx, by, chunk_rows, tiles_x, sy, vec, dst, count);
    } else if (dt == RW_F64) {
      k_gram_mfma<double, 1><<<grid, 64, 0, s>>>((const double*)X, ldx, (const double*)Y, ldy, rows, bx, by, chunk_rows, tiles_x, sy, vec, dst, count);
    } else if (dt == RW_F32) {
      k_gram_mfma<float, 1><<<grid, 64, 0, s>>>((const float*)X, ldx, (const float*)Y, ldy, rows, bx, by, chunk_rows, tiles_x, sy, vec, dst, count);
    } else {
      k_gram_mfma<uint16_t, 1><<<grid, 64, 0, s>>>((const uint16_t*)X, ldx, (const uint16_t*)Y, ldy, rows, bx, by, chunk_rows, tiles_x, sy, vec, dst, count);
    }
  } else {
    dim3 grid((bx + kGT - 1) / kGT, (by + kGT - 1) / kGT, (unsigned)nch);
    if (dt == RW_F64)
      k_gram<double><<<grid, 256, 0, s>>>((const double*)X, ldx, (const double*)Y, ldy, rows, bx, by, chunk_rows, dst, count);
    else if (dt == RW_F32)
      k_gram<float><<<grid, 256, 0, s>>>((const float*)X, ldx, (const float*)Y, ldy, rows, bx, by, chunk_rows, dst, count);
    else
      k_gram<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)X, ldx, (const uint16_t*)Y, ldy, rows, bx, by, chunk_rows, dst, count);
  }
  RW_LAUNCH_CHECK();
  if (nch > 1) {
    k_sum_chunks<<<nblocks(count, 256), 256, 0, s>>>(partial, count, nch, G);
    RW_LAUNCH_CHECK();
  }
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// Z = X V (+ beta Z): X rows x k (type T), V FP64 k x n, Z rows x n (type T).  64 x 64 output tile
// per 256-thread block, 32-wide k slabs in LDS; compute in Elem<T>::C.
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gemm(const T* X, int64_t ldx, const double* V, int64_t ldv, T* Z,
                                              int64_t ldz, int64_t rows, int k, int n, double beta) {
  using C = typename Elem<T>::C;
  __shared__ C sX[kGK][kGT + 1];   // [kk][row]
  __shared__ C sV[kGK][kGT + 1];   // [kk][col]
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kGT;
  const int c0 = blockIdx.y * kGT;
  C acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = C(0);
  for (int k0 = 0; k0 < k; k0 += kGK) {
    // X slab: 64 rows x 32 k; thread loads rows (t & 63), k-columns (t >> 6) + 4 q
    {
      int lr = threadIdx.x & 63, lk = threadIdx.x >> 6;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        int kk = lk + 4 * q;
        int64_t row = r0 + lr;
        sX[kk][lr] = (row < rows && k0 + kk < k) ? Elem<T>::ld(X, (int64_t)(k0 + kk) * ldx + row) : C(0);
      }
      int lkk = threadIdx.x & 31, lcol = threadIdx.x >> 5;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        int col = lcol + 8 * q;
        sV[lkk][col] = (k0 + lkk < k && c0 + col < n) ? (C)V[(int64_t)(c0 + col) * ldv + k0 + lkk] : C(0);
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kGK; ++kk) {
      C xv[4], vv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xv[a] = sX[kk][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) vv[b] = sV[kk][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xv[a], vv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int64_t row = r0 + tx + 16 * a;
      int col = c0 + ty + 16 * b;
      if (row < rows && col < n) {
        int64_t idx = (int64_t)col * ldz + row;
        C v = acc[a][b];
        if (beta != 0.0) v += (C)beta * Elem<T>::ld(Z, idx);
        Elem<T>::st(Z, idx, v);
      }
    }
}

// Z = X V (+ beta Z) for FP32 and BF16 X on the FP32 matrix cores (v_mfma_f32_16x16x4f32: A(i,k) from
// lane i + 16k, B(k,j) from lane j + 16k, D(4 (l/16) + v, l%16) in register v of lane l), computed as
// Z^T = V^T X^T so that a store writes 16 consecutive rows of a column per 16-lane group.  A workgroup
// keeps an FP32 copy of a slab of V's columns (all k rows) in LDS and its eight waves walk 32-row tasks;
// a wave accumulates all of the slab's 16-column blocks for its two 16-row blocks, with X fragments
// loaded four steps ahead.  Same arithmetic as the vector kernel (V rounded to FP32, FP32 accumulation).
typedef float gemm_f4 __attribute__((ext_vector_type(4)));
constexpr int kGemmWaves = 8;
constexpr int kGemmAhead = 4;   // k-steps of X loaded ahead (a step is 26 MFMAs, an HBM load some microseconds)

template <typename T, int NCB>
__global__ __launch_bounds__(64 * kGemmWaves) void k_gemm_mfma(const T* X, int64_t ldx, const double* V, int64_t ldv,
                                                               T* Z, int64_t ldz, int64_t rows, int k, int n,
                                                               double beta, int slab_w, int ld) {
  extern __shared__ float sV[];   // [kpad][ld]: V(kk, c0 + c) rounded to FP32, zero beyond k
  const int c0 = blockIdx.y * slab_w;
  const int w = std::min(slab_w, n - c0);
  const int nks = (k + 3) / 4;
  for (int t = threadIdx.x; t < 4 * nks * w; t += blockDim.x) {
    const int kk = t % (4 * nks), c = t / (4 * nks);
    sV[kk * ld + c] = kk < k ? (float)V[(int64_t)(c0 + c) * ldv + kk] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c16 = lane & 15, g = lane >> 4;
  const int64_t tasks = (rows + 31) / 32;
  for (int64_t task = (int64_t)blockIdx.x * kGemmWaves + wave; task < tasks; task += (int64_t)gridDim.x * kGemmWaves) {
    const int64_t r0 = task * 32;
    const int64_t ra = r0 + c16, rb = r0 + 16 + c16;
    const bool oa = ra < rows, ob = rb < rows;
    gemm_f4 acc[2][NCB];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[b][cb] = gemm_f4{0.f, 0.f, 0.f, 0.f};
    float xa[kGemmAhead], xb[kGemmAhead];
    auto fetch = [&](int s, float& va, float& vb) {
      const int kk = 4 * s + g;
      const bool ok = kk < k;
      va = (ok && oa) ? (float)Elem<T>::ld(X, (int64_t)kk * ldx + ra) : 0.f;
      vb = (ok && ob) ? (float)Elem<T>::ld(X, (int64_t)kk * ldx + rb) : 0.f;
    };
#pragma unroll
    for (int d = 0; d < kGemmAhead; ++d) fetch(d, xa[d], xb[d]);
    for (int s0 = 0; s0 < nks; s0 += kGemmAhead) {
#pragma unroll
      for (int d = 0; d < kGemmAhead; ++d) {
        const int s = s0 + d;
        if (s >= nks) break;
        const float fa = xa[d], fb = xb[d];
        fetch(s + kGemmAhead, xa[d], xb[d]);
        const float* vrow = sV + (4 * s + g) * ld + c16;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const float av = 16 * cb + c16 < w ? vrow[16 * cb] : 0.f;
          acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, fa, acc[0][cb], 0, 0, 0);
          acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, fb, acc[1][cb], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t row = b ? rb : ra;
      if (!(b ? ob : oa)) continue;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * cb + 4 * g + v;
          if (col >= w) continue;
          const int64_t idx = (int64_t)(c0 + col) * ldz + row;
          float out = acc[b][cb][v];
          if (beta != 0.0) out += (float)beta * (float)Elem<T>::ld(Z, idx);
          Elem<T>::st(Z, idx, out);
        }
    }
  }
}

// widest slab of V's columns whose FP32 copy fits in LDS (all columns when they fit, else a multiple of
// 16); 0 when not even 16 columns fit
static int gemm_slab_width(int k, int n) {
  const size_t kpad = (size_t)(k + 3) / 4 * 4;
  const size_t cap = kLdsLimit / (kpad * sizeof(float));
  if ((size_t)n <= cap && n <= 208) return n;
  const int w = (int)std::min<size_t>(cap, 208) / 16 * 16;
  return w;
}

template <typename T, int NCB>
static void launch_gemm_mfma(const T* X, int64_t ldx, const double* V, int64_t ldv, T* Z, int64_t ldz, int64_t rows,
                             int k, int n, double beta, int slab_w, hipStream_t s) {
  const int ld = slab_w;
  const int nslab = (n + slab_w - 1) / slab_w;
  const size_t sh = (size_t)(k + 3) / 4 * 4 * ld * sizeof(float);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_gemm_mfma<T, NCB>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
    attr = true;
  }
  const int64_t tasks = (rows + 31) / 32;
  const int64_t per = std::max<int64_t>(1, 256 / nslab);
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(per, (tasks + kGemmWaves - 1) / kGemmWaves));
  k_gemm_mfma<T, NCB><<<dim3(gx, nslab), 64 * kGemmWaves, sh, s>>>(X, ldx, V, ldv, Z, ldz, rows, k, n, beta, slab_w, ld);
}

template <typename T>
static bool gemm_mfma(const T* X, int64_t ldx, const double* V, int64_t ldv, T* Z, int64_t ldz, int64_t rows, int k,
                      int n, double beta, hipStream_t s) {
  const int sw = gemm_slab_width(k, n);
  if (sw < 16 || rows < 1024 || n < 32 || k < 16) return false;
  const int ncb = (sw + 15) / 16;
  if (ncb <= 4) launch_gemm_mfma<T, 4>(X, ldx, V, ldv, Z, ldz, rows, k, n, beta, sw, s);
  else if (ncb <= 8) launch_gemm_mfma<T, 8>(X, ldx, V, ldv, Z, ldz, rows, k, n, beta, sw, s);
  else launch_gemm_mfma<T, 13>(X, ldx, V, ldv, Z, ldz, rows, k, n, beta, sw, s);
  return true;
}

// ---------------------------------------------------------------------------------------------
// Rotation of a block with the residual norms of its operator image, in one pass (FP32 blocks):
//   X = A0 V,  LX = A1' V,  res_j = ||LX_j - theta_j X_j||,
// A1' = A1 shifted right by off1 columns (zero columns in front), so that V may carry extra leading rows
// that act on A0 only.  LX is stored only when a buffer is given.  Same arithmetic as k_gemm_mfma (V
// rounded to FP32 in LDS, FP32 accumulation); a wave walks 16-row tasks and holds both outputs'
// accumulators.  The residual terms (FP32, from the unrounded accumulators, which are the stored values)
// are summed per task over the 16 lanes of a column group, then over the wave's tasks, the waves of the
// workgroup and the workgroups, in a fixed order.  Each task reads its rows of A0 before writing its rows
// of X, so X may share A0's storage (shifted by whole columns).
// ---------------------------------------------------------------------------------------------
// sum over the 16 lanes of a DPP row (quad swaps, half-row mirror, row mirror); every lane of the row
// receives the same sum (each step adds two equal partial sums in swapped order)
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_sum(float x) {
  x += dpp_f<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += dpp_f<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += dpp_f<0x141>(x);   // row_half_mirror
  x += dpp_f<0x140>(x);   // row_mirror
  return x;
}
// four column sums over the 16 lanes of a DPP row at once (a reduce-scatter): lane i = 4 q + j of the row
// returns the sum of e[t] with t = j for even q and t = 3 - j for odd q.  The two quad steps halve the set
// of columns a lane keeps (it keeps the ones matching its t in bit 0, then in bit 1); the half-row and row
// mirrors pair lanes i and 7 - i, then i and 15 - i, which hold the same t, so that all four lanes holding
// a column end with the same sum.
__device__ __forceinline__ float row16_sum4(const float e[4], int t) {
  const bool b0 = t & 1, b1 = (t >> 1) & 1;
  const float k0 = b0 ? e[1] : e[0], k1 = b0 ? e[3] : e[2];
  const float s0 = b0 ? e[0] : e[1], s1 = b0 ? e[2] : e[3];
  const float a0 = k0 + dpp_f<0xB1>(s0), a1 = k1 + dpp_f<0xB1>(s1);   // columns (t & 1) and (t & 1) + 2
  float b = (b1 ? a1 : a0) + dpp_f<0x4E>(b1 ? a0 : a1);               // column t, over the quad
  b += dpp_f<0x141>(b);
  b += dpp_f<0x140>(b);
  return b;
}

constexpr int kRotAhead = 2;   // k-steps of the two inputs loaded ahead (two outputs' accumulators held)

// number of 16-column groups the rotation kernel is instantiated for (n columns)
static inline int rot_ncb(int n) {
  const int ncb = (n + 15) / 16;
  return ncb <= 4 ? 4 : (ncb <= 8 ? 8 : 13);
}

template <int NCB>
__global__ __launch_bounds__(64 * kGemmWaves) void k_rotate_pair(const float* A0, const float* A1, int off1,
                                                                 int64_t ld, const double* V, int64_t ldv,
                                                                 const double* theta, float* X, float* LX,
                                                                 int64_t rows, int k, int n, double* rpart) {
  extern __shared__ float sV[];   // [kpad][n] V rounded to FP32 (zero beyond k), then theta (zero beyond n)
  const int nks = (k + 3) / 4;
  for (int t = threadIdx.x; t < 4 * nks * n; t += blockDim.x) {
    const int kk = t % (4 * nks), c = t / (4 * nks);
    sV[kk * n + c] = kk < k ? (float)V[(int64_t)c * ldv + kk] : 0.f;
  }
  float* sTh = sV + 4 * nks * n;   // 16-byte aligned (4 nks n floats)
  for (int c = threadIdx.x; c < 16 * NCB; c += blockDim.x) sTh[c] = c < n ? (float)theta[c] : 0.f;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c16 = lane & 15, g = lane >> 4;
  // lane c16 keeps the residual sums of columns 16 cb + 4 g + t (see row16_sum4)
  const int t = ((c16 >> 2) & 1) ? 3 - (c16 & 3) : (c16 & 3);
  float rps[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) rps[cb] = 0.f;
  const int64_t tasks = (rows + 15) / 16;
  for (int64_t task = (int64_t)blockIdx.x * kGemmWaves + wave; task < tasks; task += (int64_t)gridDim.x * kGemmWaves) {
    const int64_t r = task * 16 + c16;
    const bool ok = r < rows;
    gemm_f4 acc0[NCB], acc1[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      acc0[cb] = gemm_f4{0.f, 0.f, 0.f, 0.f};
      acc1[cb] = gemm_f4{0.f, 0.f, 0.f, 0.f};
    }
    float x0[kRotAhead], x1[kRotAhead];
    auto fetch = [&](int st, float& a, float& b) {
      const int kk = 4 * st + g;
      a = (ok && kk < k) ? A0[(int64_t)kk * ld + r] : 0.f;
      b = (ok && kk < k && kk >= off1) ? A1[(int64_t)(kk - off1) * ld + r] : 0.f;
    };
#pragma unroll
    for (int d = 0; d < kRotAhead; ++d) fetch(d, x0[d], x1[d]);
    for (int s0 = 0; s0 < nks; s0 += kRotAhead) {
#pragma unroll
      for (int d = 0; d < kRotAhead; ++d) {
        const int st = s0 + d;
        if (st >= nks) break;
        const float fa = x0[d], fb = x1[d];
        fetch(st + kRotAhead, x0[d], x1[d]);
        const float* vrow = sV + (4 * st + g) * n + c16;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const float av = 16 * cb + c16 < n ? vrow[16 * cb] : 0.f;
          acc0[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, fa, acc0[cb], 0, 0, 0);
          acc1[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, fb, acc1[cb], 0, 0, 0);
        }
      }
    }
    // the lane's output columns 16 cb + 4 g + v by a running offset (column steps of 1 and 13)
    int64_t off = (int64_t)(4 * g) * ld + r;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      if (16 * cb >= n) break;   // uniform
      const gemm_f4 th = *reinterpret_cast<const gemm_f4*>(sTh + 16 * cb + 4 * g);
      float e[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * cb + 4 * g + v;
        e[v] = 0.f;
        if (ok && col < n) {
          const float xv = acc0[cb][v], lv = acc1[cb][v];
          X[off] = xv;
          if (LX) LX[off] = lv;
          const float dv = lv - th[v] * xv;
          e[v] = dv * dv;
        }
        off += v < 3 ? ld : 13 * ld;
      }
      rps[cb] += row16_sum4(e, t);
    }
  }
  // column sums over the waves (in order), then one value per workgroup
  __syncthreads();   // V no longer read
  double* red = reinterpret_cast<double*>(sV);   // [kGemmWaves][n]
  if (c16 < 4) {   // quad 0: t = c16
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int col = 16 * cb + 4 * g + c16;
      if (col < n) red[wave * n + col] = (double)rps[cb];
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < kGemmWaves; ++w) s += red[w * n + c];
    rpart[(int64_t)blockIdx.x * n + c] = s;
  }
}

// one wave per column: lanes take every 64th workgroup's value, then a butterfly (fixed order)
__global__ __launch_bounds__(64) void k_rotate_res_final(const double* rpart, int nblk, int n, double* res) {
  const int c = blockIdx.x, lane = threadIdx.x;
  double t = 0.0;
  for (int b = lane; b < nblk; b += 64) t += rpart[(int64_t)b * n + c];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
  if (lane == 0) res[c] = sqrt(t);
}

static size_t rotate_pair_lds(int k, int n) {
  const size_t nks = (size_t)(k + 3) / 4;
  return (4 * nks * n + 16 * (size_t)rot_ncb(n)) * sizeof(float);
}

bool rotate_pair_fits(int dt, int64_t rows, int k, int n) {
  return dt == RW_F32 && rows >= 1024 && n >= 32 && n <= 208 && k >= 16 && rotate_pair_lds(k, n) <= kLdsLimit &&
         (size_t)kGemmWaves * n * sizeof(double) <= rotate_pair_lds(k, n);
}

size_t rotate_pair_partial_count(int n) { return (size_t)256 * n; }

template <int NCB>
static void launch_rotate_pair(const float* A0, const float* A1, int off1, int64_t ld, const double* V, int64_t ldv,
                               const double* theta, float* X, float* LX, int64_t rows, int k, int n, double* res,
                               double* partial, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_rotate_pair<NCB>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
    attr = true;
  }
  const int64_t tasks = (rows + 15) / 16;
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(256, (tasks + kGemmWaves - 1) / kGemmWaves));
  k_rotate_pair<NCB><<<gx, 64 * kGemmWaves, rotate_pair_lds(k, n), s>>>(A0, A1, off1, ld, V, ldv, theta, X, LX, rows,
                                                                        k, n, partial);
  k_rotate_res_final<<<n, 64, 0, s>>>(partial, (int)gx, n, res);
}

int rotate_pair(const float* A0, const float* A1, int off1, int64_t ld, const double* V, int64_t ldv,
                const double* theta, float* X, float* LX, int64_t rows, int k, int n, double* res, double* partial,
                hipStream_t s) {
  RW_CHECK(rotate_pair_fits(RW_F32, rows, k, n) && (off1 == 0 || off1 == 1), RW_EINVAL, "rotate_pair: bad shape");
  const int ncb = rot_ncb(n);
  if (ncb == 4) launch_rotate_pair<4>(A0, A1, off1, ld, V, ldv, theta, X, LX, rows, k, n, res, partial, s);
  else if (ncb == 8) launch_rotate_pair<8>(A0, A1, off1, ld, V, ldv, theta, X, LX, rows, k, n, res, partial, s);
  else launch_rotate_pair<13>(A0, A1, off1, ld, V, ldv, theta, X, LX, rows, k, n, res, partial, s);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

bool gemm_rowwise(int dt, int64_t rows, int k, int n) {
  if (dt != RW_F32 && dt != RW_BF16) return false;
  const int sw = gemm_slab_width(k, n);
  return sw >= n && sw >= 16 && rows >= 1024 && n >= 32 && k >= 16;
}

int gemm_tn(int dt, const void* X, int64_t ldx, const double* V, int64_t ldv, void* Z, int64_t ldz,
            int64_t rows, int k, int n, double beta, hipStream_t s) {
  if (rows <= 0 || n <= 0) return RW_OK;
  if (dt == RW_F32 && gemm_mfma((const float*)X, ldx, V, ldv, (float*)Z, ldz, rows, k, n, beta, s)) {
    RW_LAUNCH_CHECK();
    return RW_OK;
  }
  if (dt == RW_BF16 && gemm_mfma((const uint16_t*)X, ldx, V, ldv, (uint16_t*)Z, ldz, rows, k, n, beta, s)) {
    RW_LAUNCH_CHECK();
    return RW_OK;
  }
  dim3 grid((unsigned)((rows + kGT - 1) / kGT), (n + kGT - 1) / kGT);
  if (dt == RW_F64)
    k_gemm<double><<<grid, 256, 0, s>>>((const double*)X, ldx, V, ldv, (double*)Z, ldz, rows, k, n, beta);
  else if (dt == RW_F32)
    k_gemm<float><<<grid, 256, 0, s>>>((const float*)X, ldx, V, ldv, (float*)Z, ldz, rows, k, n, beta);
  else
    k_gemm<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)X, ldx, V, ldv, (uint16_t*)Z, ldz, rows, k, n, beta);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------------------------
template <typename S, typename D>
__global__ void k_convert(const S* src, int64_t lds, D* dst, int64_t ldd, int64_t rows, int cols) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  if (r >= rows || c >= cols) return;
  typename Elem<S>::C v = Elem<S>::ld(src, (int64_t)c * lds + r);
  Elem<D>::st(dst, (int64_t)c * ldd + r, (typename Elem<D>::C)v);
}

template <typename S>
static int convert_from(const S* src, int64_t lds, int dt_dst, void* dst, int64_t ldd, int64_t rows, int cols,
                        hipStream_t s) {
  dim3 grid(nblocks(rows, 256), cols);
  if (dt_dst == RW_F64) k_convert<S, double><<<grid, 256, 0, s>>>(src, lds, (double*)dst, ldd, rows, cols);
  else if (dt_dst == RW_F32) k_convert<S, float><<<grid, 256, 0, s>>>(src, lds, (float*)dst, ldd, rows, cols);
  else k_convert<S, uint16_t><<<grid, 256, 0, s>>>(src, lds, (uint16_t*)dst, ldd, rows, cols);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

int convert_block(int dt_src, const void* src, int64_t lds, int dt_dst, void* dst, int64_t ldd, int64_t rows,
                  int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return RW_OK;
  RW_CHECK(cols <= 65535, RW_EINVAL, "too many columns to convert");
  if (dt_src == RW_F64) return convert_from((const double*)src, lds, dt_dst, dst, ldd, rows, cols, s);
  if (dt_src == RW_F32) return convert_from((const float*)src, lds, dt_dst, dst, ldd, rows, cols, s);
  return convert_from((const uint16_t*)src, lds, dt_dst, dst, ldd, rows, cols, s);
}

// pair form: thread (r, c) writes hi = bf16(q_c) to column kPairCols + c and, for 1 <= c <= kPairCols, the
// remainder bf16(q_c - hi) (formed in the source precision) to column c - 1; column c = 0 also zeroes the
// remainder columns of q_j with j >= cols
template <typename S>
__global__ void k_convert_pair(const S* src, int64_t rows, int cols, uint16_t* dst) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= rows || c >= cols) return;
  const S v = src[(int64_t)c * rows + r];
  const uint16_t hi = f32_to_bf16((float)v);
  dst[(int64_t)(kPairCols + c) * rows + r] = hi;
  if (c >= 1 && c <= kPairCols) dst[(int64_t)(c - 1) * rows + r] = f32_to_bf16((float)(v - (S)bf16_to_f32(hi)));
  if (c == 0)
    for (int j = cols > 1 ? cols : 1; j <= kPairCols; ++j) dst[(int64_t)(j - 1) * rows + r] = 0;
}

int convert_pair(int dt_src, const void* src, int64_t rows, uint16_t* dst, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return RW_OK;
  RW_CHECK(cols <= 65535, RW_EINVAL, "too many columns to convert");
  const dim3 grid(nblocks(rows, 256), cols);
  if (dt_src == RW_F64) k_convert_pair<double><<<grid, 256, 0, s>>>((const double*)src, rows, cols, dst);
  else k_convert_pair<float><<<grid, 256, 0, s>>>((const float*)src, rows, cols, dst);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// residual norms ||A_j - theta_j B_j|| in FP64, deterministic (per-column block partials)
// ---------------------------------------------------------------------------------------------
constexpr int kNormChunks = 64;

template <typename T>
__global__ void k_colnorm_partial(const T* A, const T* B, const double* theta, int64_t rows, int64_t ld,
                                  double* partial) {
  const int col = blockIdx.y;
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * per, r1 = std::min<int64_t>(rows, r0 + per);
  double th = theta ? theta[col] : 0.0;
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    double v = (double)Elem<T>::ld(A, (int64_t)col * ld + r);
    if (theta) v -= th * (double)Elem<T>::ld(B, (int64_t)col * ld + r);
    acc += v * v;
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)col * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void k_colnorm_final(const double* partial, int nchunks, int cols, double* out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int k = 0; k < nchunks; ++k) s += partial[(int64_t)c * nchunks + k];
  out[c] = sqrt(s);
}

int residual_norms(int dt, const void* A, const void* B, const double* theta, int64_t rows, int cols, int64_t ld,
                   double* out, double* partial, hipStream_t s) {
  if (cols <= 0) return RW_OK;
  RW_CHECK(cols <= 65535, RW_EINVAL, "too many columns");
  dim3 grid(kNormChunks, cols);
  if (dt == RW_F64) k_colnorm_partial<double><<<grid, 256, 0, s>>>((const double*)A, (const double*)B, theta, rows, ld, partial);
  else if (dt == RW_F32) k_colnorm_partial<float><<<grid, 256, 0, s>>>((const float*)A, (const float*)B, theta, rows, ld, partial);
  else k_colnorm_partial<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)A, (const uint16_t*)B, theta, rows, ld, partial);
  RW_LAUNCH_CHECK();
  k_colnorm_final<<<nblocks(cols, 256), 256, 0, s>>>(partial, kNormChunks, cols, out);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

size_t norm_partial_count(int cols) { return (size_t)kNormChunks * cols; }

// ---------------------------------------------------------------------------------------------
// random start block: standard normals from a counter-based generator (splitmix64 of the element
// index and seed, then Box-Muller), identical on every launch for the same seed
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void k_fill_random(T* X, int64_t ld, int64_t rows, int cols, uint64_t seed) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  if (r >= rows) return;
  uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)c * 0x100000001b3ull + (uint64_t)r));
  double u1 = ((h >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
  uint64_t h2 = splitmix64(h);
  double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);          // [0, 1)
  double v = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  Elem<T>::st(X, (int64_t)c * ld + r, (typename Elem<T>::C)v);
}

int fill_random(int dt, void* X, int64_t ld, int64_t rows, int cols, uint64_t seed, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return RW_OK;
  dim3 grid(nblocks(rows, 256), cols);
  if (dt == RW_F64) k_fill_random<double><<<grid, 256, 0, s>>>((double*)X, ld, rows, cols, seed);
  else if (dt == RW_F32) k_fill_random<float><<<grid, 256, 0, s>>>((float*)X, ld, rows, cols, seed);
  else k_fill_random<uint16_t><<<grid, 256, 0, s>>>((uint16_t*)X, ld, rows, cols, seed);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// X -= v (v^T X) for a unit vector v
// ---------------------------------------------------------------------------------------------
int project_out_to(int dt, const void* X, int64_t ldx, void* Y, int64_t ldy, const void* v, int64_t rows, int cols,
                   double* tmp, double* partial, hipStream_t s);
// d_j = v^T X_j for one vector v (the 1 x cols Gram): block (j, chunk) reduces its rows in a fixed order
// (strided per-thread sums, then a tree in LDS); FP64 accumulation.  HBM-bound: X is read once.
template <typename T>
__global__ __launch_bounds__(256) void k_vdot_cols(const T* v, const T* X, int64_t ld, int64_t rows,
                                                   int64_t chunk_rows, int cols, double* out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const int64_t r0 = blockIdx.y * chunk_rows;
  const int64_t r1 = std::min<int64_t>(rows, r0 + chunk_rows);
  const T* xj = X + (int64_t)j * ld;
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256)
    acc += (double)Elem<T>::ld(v, r) * (double)Elem<T>::ld(xj, r);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)blockIdx.y * cols + j] = red[0];
}

static int vdot_cols(int dt, const void* v, const void* X, int64_t ld, int64_t rows, int cols, double* d,
                     double* partial, hipStream_t s) {
  int64_t nch = gram_chunks(rows, 1, cols);        // the partial buffer holds nch x cols values
  int64_t chunk_rows = (rows + nch - 1) / nch;
  nch = (rows + chunk_rows - 1) / chunk_rows;
  double* dst = nch == 1 ? d : partial;
  dim3 grid(cols, (unsigned)nch);
  if (dt == RW_F64) k_vdot_cols<double><<<grid, 256, 0, s>>>((const double*)v, (const double*)X, ld, rows, chunk_rows, cols, dst);
  else if (dt == RW_F32) k_vdot_cols<float><<<grid, 256, 0, s>>>((const float*)v, (const float*)X, ld, rows, chunk_rows, cols, dst);
  else k_vdot_cols<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)v, (const uint16_t*)X, ld, rows, chunk_rows, cols, dst);
  RW_LAUNCH_CHECK();
  if (nch > 1) {
    k_sum_chunks<<<nblocks(cols, 256), 256, 0, s>>>(partial, cols, nch, d);
    RW_LAUNCH_CHECK();
  }
  return RW_OK;
}

int project_out(int dt, void* X, int64_t ld, const void* v, int64_t rows, int cols, double* tmp, double* partial,
                hipStream_t s) {
  return project_out_to(dt, X, ld, X, ld, v, rows, cols, tmp, partial, s);
}

// Y = X - v (v^T X): the same two passes, reading X and writing Y (Y may be X)
template <typename T>
__global__ void k_rank1_sub_to(const T* X, int64_t ldx, T* Y, int64_t ldy, const T* v, const double* t, int64_t rows,
                               int cols) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= rows) return;
  using C = typename Elem<T>::C;
  const C val = Elem<T>::ld(X, (int64_t)c * ldx + r) - (C)t[c] * Elem<T>::ld(v, r);
  Elem<T>::st(Y, (int64_t)c * ldy + r, val);
}

int project_out_to(int dt, const void* X, int64_t ldx, void* Y, int64_t ldy, const void* v, int64_t rows, int cols,
                   double* tmp, double* partial, hipStream_t s) {
  if (cols <= 0) return RW_OK;
  RW_TRY(vdot_cols(dt, v, X, ldx, rows, cols, tmp, partial, s));
  dim3 grid(nblocks(rows, 256), cols);
  if (dt == RW_F64)
    k_rank1_sub_to<double><<<grid, 256, 0, s>>>((const double*)X, ldx, (double*)Y, ldy, (const double*)v, tmp, rows, cols);
  else if (dt == RW_F32)
    k_rank1_sub_to<float><<<grid, 256, 0, s>>>((const float*)X, ldx, (float*)Y, ldy, (const float*)v, tmp, rows, cols);
  else
    k_rank1_sub_to<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)X, ldx, (uint16_t*)Y, ldy, (const uint16_t*)v, tmp,
                                                   rows, cols);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // namespace rw

namespace rw {

// ---------------------------------------------------------------------------------------------
// column dot products d_j = a_j^T b_j in FP64 (deterministic per-column partials)
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_coldot_partial(const T* A, const T* B, int64_t rows, int64_t ld, double* partial) {
  const int col = blockIdx.y;
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * per, r1 = std::min<int64_t>(rows, r0 + per);
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x)
    acc += (double)Elem<T>::ld(A, (int64_t)col * ld + r) * (double)Elem<T>::ld(B, (int64_t)col * ld + r);
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)col * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void k_coldot_final(const double* partial, int nchunks, int cols, double* out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int k = 0; k < nchunks; ++k) s += partial[(int64_t)c * nchunks + k];
  out[c] = s;
}

int col_dots(int dt, const void* A, const void* B, int64_t rows, int cols, int64_t ld, double* out, double* partial,
             hipStream_t s) {
  if (cols <= 0) return RW_OK;
  RW_CHECK(cols <= 65535, RW_EINVAL, "too many columns");
  dim3 grid(kNormChunks, cols);
  if (dt == RW_F64) k_coldot_partial<double><<<grid, 256, 0, s>>>((const double*)A, (const double*)B, rows, ld, partial);
  else if (dt == RW_F32) k_coldot_partial<float><<<grid, 256, 0, s>>>((const float*)A, (const float*)B, rows, ld, partial);
  else k_coldot_partial<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)A, (const uint16_t*)B, rows, ld, partial);
  RW_LAUNCH_CHECK();
  k_coldot_final<<<nblocks(cols, 256), 256, 0, s>>>(partial, kNormChunks, cols, out);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// max |x_i| over a vector (single block, fixed order)
__global__ void k_absmax(const double* x, int64_t n, double* out) {
  __shared__ double sh[1024];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, fabs(x[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

int absmax(const double* x, int64_t n, double* out, hipStream_t s) {
  k_absmax<<<1, 1024, 0, s>>>(x, n, out);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // namespace rw
