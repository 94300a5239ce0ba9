// Online random-walker solve in the precomputed eigenbasis (Sec. II-B eqs. (7)-(17); the gamma = 0
// case after eq. (17)) and the seed-driven choice of m (Sec. III-A1 eq. (24)).
//
// Reduced system.  With the null vector as Q's column 0 (eigenvalue 0), the gamma = 0 bordered seed
// system in (F_s, c) is equivalent to an m x m system in the coefficients Y of U_hat_n = Q_n Y:
// the ansatz gives F_s = op_ss U_hat_s + B Q_n Y, and the conditions Q'_s^T F_s = Lambda' Y' (from
// U_n = R^T F_s + g_n c^T) and g_s^T F_s = 0 (from g^T F = 0, F_n = 0) are the rows of
//     (Lambda - Q_s^T B Q_n) Y = Q_s^T op_ss U_hat_s.
// Its size is m, not S, and Lambda enters without inversion, so near-null eigenvalues need no
// clamping.  The reconstruction U = D^{-1/2} Q Y is one tall-skinny pass over Q.
//
// Precision.  A weakly coupled graph (two regions joined by weights near the FP64 underflow of the
// exponent) has a second near-null pair, and the reduced matrix then has a condition number near 1/u:
// its near-singular rows are formed by cancellation, and the rounding of an FP32 coefficient, or of an
// FP32 null vector stored as Q's column 0, decides the solution there.  So the seed rows are formed from
// the FP64 weights and degrees, and after m is chosen the basis is taken in FP64 as the exact null vector
// g plus the stored columns made orthogonal to it (q'_j = (q_j - g c_j) / n_j, c_j = g^T q_j): one pass
// over Q's first m columns gives the c_j and n_j, the seed rows are corrected in place, and the
// reconstruction reads columns 1..m-1 with the null vector's term as a per-label constant (s_i g_i is the
// same on every node with d_i > 0).  The choice of m fits the stored columns as they are.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "rw_internal.h"

namespace rw {

// candidate m values evaluated per probe of the choice of m: all of [2, m_avail] at once when
// m_avail <= 256 (one batched launch), else a k-ary search
static inline int fit_cands(int ma) { return std::max(1, std::min(ma - 1, 256)); }

struct SolveWork {
  uint8_t* map;       // N: 0 = not a seed, else label + 1
  uint8_t* anc;       // N: anchoring check scratch
  int64_t* seeds;     // S
  int32_t* labels;    // S
  double* Qs;         // S x ma   (seed rows of Q)
  double* GB;         // S x ma   (B Q_n)
  double* Hs;         // S x C    (op_ss U_hat_s)
  double* Us;         // S x C    (U_hat_s)
  double* gs;         // S        (g at the seeds, FP64)
  double* Bg;         // S        (B g_n)
  double* cn;         // 2 ma     (c_j, n_j of the FP64 basis)
  double* npart;      // null_stats partials
  int* nbad;          // set when some n_j is not positive
  double* Gq;         // ma x ma  (Q_s^T Q_s)
  double* Gb;         // ma x C   (Q_s^T U_hat_s)
  double* fvals;      // ncand x C
  double* fitA;       // ncand x ms x ms  (ms = min(S, ma))
  double* fitR;       // ncand x ms x C
  double* fitW;       // ncand x ms
  double* fitWork;    // eigensolver work (Jacobi, or the batched tridiagonal solver)
  size_t fitWorkCount;
  double* K;          // ma x ma
  double* Y;          // ma x C
  double* stat;       // 8
  double* partial;
  double* scrF;       // (ma + 1): max over labels of the least-squares residual at m
  int* scrCls;        // (ma + 1): 0 fails, 1 passes, 2 undecided; [0] = factorized leading size
};

// fit = false leaves out the choice-of-m arrays (solves with a fixed m)
static size_t solve_layout(const Graph* g, int ma, int64_t S, int C, void* base, SolveWork* w, bool fit = true) {
  Carver c(base);
  int64_t ms = std::min<int64_t>(S, ma);
  SolveWork t;
  t.map = c.take<uint8_t>(g->N);
  t.anc = c.take<uint8_t>(g->N);
  t.seeds = c.take<int64_t>(S);
  t.labels = c.take<int32_t>(S);
  t.Qs = c.take<double>(S * ma);
  t.GB = c.take<double>(S * ma);
  t.Hs = c.take<double>(S * C);
  t.Us = c.take<double>(S * C);
  t.gs = c.take<double>(S);
  t.Bg = c.take<double>(S);
  t.cn = c.take<double>(2 * (size_t)ma);
  t.npart = c.take<double>(null_stats_partial_count(g->N, ma));
  t.Gq = c.take<double>((size_t)ma * ma);
  t.Gb = c.take<double>((size_t)ma * C);
  const int nc = fit ? fit_cands(ma) : 0;
  t.fvals = c.take<double>((size_t)nc * C);
  t.fitA = c.take<double>((size_t)nc * ms * ms);
  t.fitR = c.take<double>((size_t)nc * ms * C);
  t.fitW = c.take<double>((size_t)nc * ms);
  t.fitWorkCount = fit ? syev_work_count((int)ms, nc, false, C) : 0;
  if (fit && tridiag_batch_fits((int)ms))
    t.fitWorkCount = std::max(t.fitWorkCount, tridiag_rhs_work_count((int)ms, std::min(nc, kTriBatchMax), C));
  t.fitWork = c.take<double>(t.fitWorkCount);
  t.K = c.take<double>((size_t)ma * ma);
  t.Y = c.take<double>((size_t)ma * C);
  t.stat = c.take<double>(8);
  t.nbad = c.take<int>(4);   // after stat: the two are read back with one copy
  size_t pc = std::max(gram_partial_count(S, ma, ma), gram_partial_count(S, ma, C));
  t.partial = c.take<double>(pc);
  t.scrF = c.take<double>((size_t)ma + 1);
  t.scrCls = c.take<int>((size_t)ma + 1);
  if (w) *w = t;
  return c.used;
}

// ---------------------------------------------------------------------------------------------
// seed bookkeeping
// ---------------------------------------------------------------------------------------------
__global__ void k_clear_map(uint8_t* map, int64_t N) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) map[i] = 0;
}

__global__ void k_set_map(uint8_t* map, const int64_t* seeds, const int32_t* labels, int64_t S) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < S) map[seeds[k]] = (uint8_t)(labels[k] + 1);
}

// One block per seed: the stored columns at the seed row, B Q_n, U_hat_s, op_ss U_hat_s, g and B g_n, from the
// FP64 weights and degrees (gather_seed_row).
template <typename TQ>
__global__ void k_seed_gather(GridDev G, int normalized, const TQ* Q, const TQ* Qlo, int ma, const int64_t* seeds,
                              const uint8_t* map, const double* weight, const double* degree, const double* sums,
                              int64_t S, int C, double* Qs, double* GB, double* Hs, double* Us, double* gs, double* Bg) {
  const int64_t k = blockIdx.x;
  gather_seed_row<TQ>(G, normalized, weight, degree, sums, Q, Qlo, ma, map, seeds[k], C, nullptr, k, S, Qs, GB, Hs,
                      Us, gs, Bg);
}

// seed rows of the FP64 basis: column 0 becomes g, the others (q_j - g c_j) / n_j (in place, first m columns)
__global__ void k_seed_correct(double* Qs, double* GB, const double* gs, const double* Bg, const double* cn, int64_t S,
                               int m) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= S * m) return;
  const int64_t k = t % S;
  const int j = (int)(t / S);
  if (j == 0) {
    Qs[t] = gs[k];
    GB[t] = Bg[k];
  } else {
    const double c = cn[j], n = cn[m + j];
    Qs[t] = (Qs[t] - gs[k] * c) / n;
    GB[t] = (GB[t] - Bg[k] * c) / n;
  }
}

// ---------------------------------------------------------------------------------------------
// c_j = g^T q_j and ||q_j||^2 for j in [1, m): blocks over (2048-row chunk, 8 columns); each thread issues
// all 64 loads of its eight rows x eight columns before any reduction, sums in FP64 (products of FP32 or
// BF16 values are exact), then 16 wave sums by DPP and the four waves in order; per column, one wave sums
// the chunk partials (fixed order, so the result does not depend on the launch).
// ---------------------------------------------------------------------------------------------
constexpr int kNsRowsPerThread = 8;
constexpr int kNsRows = 256 * kNsRowsPerThread;
constexpr int kNsCols = 8;

size_t null_stats_partial_count(int64_t N, int m) {
  return (size_t)2 * m * (size_t)((N + kNsRows - 1) / kNsRows);
}

static_assert(kNsCols == kPairCols, "the first column block holds exactly the pair form's remainder columns");

// Qlo: the pair form's remainder columns (or null), added to columns 1 .. kPairCols (block row 0)
template <typename TQ>
__global__ __launch_bounds__(256) void k_null_stats(const TQ* Q, const TQ* Qlo, int64_t N, int m,
                                                    const double* degree, int normalized, double* partial,
                                                    int64_t nchunk) {
  __shared__ double sh[4][2 * kNsCols];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t chunk = blockIdx.x;
  const int j0 = 1 + (int)blockIdx.y * kNsCols;
  const int ncol = min(kNsCols, m - j0);   // >= 1, uniform
  const int64_t r0 = chunk * kNsRows + tid;
  // clamped rows and columns keep every load unconditional (straight-line code, all loads in flight);
  // rows past N carry weight 0, columns past m - 1 are read again and not stored
  int64_t ic[kNsRowsPerThread];
  double msk[kNsRowsPerThread];
#pragma unroll
  for (int q = 0; q < kNsRowsPerThread; ++q) {
    const int64_t i = r0 + 256 * q;
    ic[q] = i < N ? i : N - 1;
    msk[q] = i < N ? 1.0 : 0.0;
  }
  double v[kNsCols][kNsRowsPerThread];
#pragma unroll
  for (int jj = 0; jj < kNsCols; ++jj) {
    const TQ* qc = Q + (int64_t)(j0 + min(jj, ncol - 1)) * N;
#pragma unroll
    for (int q = 0; q < kNsRowsPerThread; ++q) v[jj][q] = (double)Elem<TQ>::ld(qc, ic[q]);
  }
  if (Qlo != nullptr && blockIdx.y == 0) {   // uniform per block
#pragma unroll
    for (int jj = 0; jj < kNsCols; ++jj) {
      const TQ* lc = Qlo + (int64_t)min(jj, ncol - 1) * N;
#pragma unroll
      for (int q = 0; q < kNsRowsPerThread; ++q) v[jj][q] += (double)Elem<TQ>::ld(lc, ic[q]);
    }
  }
  double sd[kNsRowsPerThread];
#pragma unroll
  for (int q = 0; q < kNsRowsPerThread; ++q) sd[q] = msk[q] * (normalized ? sqrt(degree[ic[q]]) : 1.0);
#pragma unroll
  for (int jj = 0; jj < kNsCols; ++jj) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int q = 0; q < kNsRowsPerThread; ++q) {
      a += sd[q] * v[jj][q];
      b += msk[q] * (v[jj][q] * v[jj][q]);
    }
    a = wave_sum64(a);
    b = wave_sum64(b);
    if (lane == 0) {
      sh[wave][2 * jj] = a;
      sh[wave][2 * jj + 1] = b;
    }
  }
  __syncthreads();
  if (tid < 2 * ncol) {
    const int j = j0 + tid / 2;
    const double t = (sh[0][tid] + sh[1][tid]) + (sh[2][tid] + sh[3][tid]);
    partial[((int64_t)j * 2 + (tid & 1)) * nchunk + chunk] = t;
  }
}

// one wave per column j >= 1 (block j - 1): lanes take the chunk partials in strides, then a wave sum
__global__ __launch_bounds__(64) void k_null_finish(const double* partial, int64_t nchunk, int m, const double* sums,
                                                    int normalized, int64_t N, double* cn, int* bad) {
  const int j = 1 + blockIdx.x;
  const int lane = threadIdx.x;
  const double* pa = partial + (int64_t)j * 2 * nchunk;
  const double* pb = pa + nchunk;
  double a = 0.0, b = 0.0;
  for (int64_t q = lane; q < nchunk; q += 64) {
    a += pa[q];
    b += pb[q];
  }
  a = wave_sum64(a);
  b = wave_sum64(b);
  if (lane == 0) {
    // g = D^{1/2} 1 / sqrt(1^T D 1) (or 1 / sqrt(N)): c_j = (sum_i d_i^{1/2} q_ij) / sqrt(1^T D 1)
    const double c = a / sqrt(normalized ? sums[0] : (double)N);
    const double n2 = b - c * c;
    cn[j] = c;
    cn[m + j] = n2 > 0.0 ? sqrt(n2) : 1.0;
    if (!(n2 > 0.0)) *bad = j;
    if (j == 1) {
      cn[0] = 0.0;
      cn[m] = 1.0;
    }
  }
}

int null_stats(const Graph* g, const void* Q, int qdt, int m, double* partial, double* cn, int* bad, hipStream_t s) {
  const int64_t nchunk = (g->N + kNsRows - 1) / kNsRows;
  const BasisView b = basis_view(g->N, Q, qdt);
  if (m > 1) {
    const dim3 grid((unsigned)nchunk, (unsigned)((m - 1 + kNsCols - 1) / kNsCols));
    if (b.dt == RW_F64)
      k_null_stats<double><<<grid, 256, 0, s>>>((const double*)b.hi, nullptr, g->N, m, g->degree, g->normalized,
                                                 partial, nchunk);
    else if (b.dt == RW_F32)
      k_null_stats<float><<<grid, 256, 0, s>>>((const float*)b.hi, nullptr, g->N, m, g->degree, g->normalized,
                                                partial, nchunk);
    else
      k_null_stats<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)b.hi, b.lo, g->N, m, g->degree, g->normalized,
                                                   partial, nchunk);
    RW_LAUNCH_CHECK();
  }
  if (m > 1) {
    k_null_finish<<<m - 1, 64, 0, s>>>(partial, nchunk, m, g->sums, g->normalized, g->N, cn, bad);
    RW_LAUNCH_CHECK();
  }
  return RW_OK;
}

__global__ __launch_bounds__(256) void k_solve_coeffs(double* Y, int m, int C, const double* cn, const double* sums,
                                                      int normalized, int64_t N) {
  solve_coeffs_block(Y, m, C, cn, ghat_scaled64(sums, normalized, N));
}

int solve_coeffs(double* Y, int m, int C, const double* cn, const Graph* g, hipStream_t s) {
  k_solve_coeffs<<<1, 256, 0, s>>>(Y, m, C, cn, g->sums, g->normalized, g->N);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

__global__ __launch_bounds__(256) void k_reduced(int m, int C, int64_t S, const double* Qs, const double* GB,
                                                 const double* Hs, const double* lambda, double gamma, double* K,
                                                 double* Y) {
  __shared__ double sA[kRedTile * 33], sB[kRedTile * 33];
  reduced_tile(blockIdx.x, blockIdx.y, m, C, S, S, Qs, GB, Hs, lambda, gamma, K, Y, sA, sB);
}

static dim3 reduced_grid(int m, int C) {
  return dim3((unsigned)((m + kRedTile - 1) / kRedTile), (unsigned)((m + C + kRedTile - 1) / kRedTile));
}


// ---------------------------------------------------------------------------------------------
// reconstruction: U(lab, i) = s_i * sum_{j>=1} Q(i, j) Y(j, lab) + kappa_lab on non-seeds (s = d^{-1/2} or 1;
// kappa = Y(0, lab), the null vector's term, added where s_i > 0 or the operator is L), one-hot on seeds.
// Y (rows 1..m-1) and kappa live in LDS; each thread owns one node and CB labels.
// ---------------------------------------------------------------------------------------------
// Qlo (the pair form's remainder columns of q_1 .. q_pm, or null) adds its terms after the plain block's.
template <typename TQ, typename TU, int CB>
__global__ __launch_bounds__(256) void k_reconstruct(const TQ* Q, const TQ* Qlo, int pm, int64_t N, int m,
                                                      const double* Y, int C, int lab0, const uint8_t* map,
                                                      const TU* dinv, int normalized, TU* U) {
  using CT = typename Elem<TQ>::C;
  extern __shared__ char smem[];
  CT* sY = reinterpret_cast<CT*>(smem);          // (m - 1) x CB
  CT* sK = sY + (m - 1) * CB;                     // CB
  for (int t = threadIdx.x; t < m * CB; t += blockDim.x) {
    int j = t / CB, c = t % CB;
    int lab = lab0 + c;
    const CT v = lab < C ? (CT)Y[j + (int64_t)lab * m] : CT(0);
    if (j == 0) sK[c] = v;
    else sY[(j - 1) * CB + c] = v;
  }
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const TQ* Q1 = Q + N;   // columns 1 .. m-1
  const int mq = m - 1;
  CT acc[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) acc[c] = CT(0);
  int j = 0;
  for (; j + 4 <= mq; j += 4) {
    CT q0 = Elem<TQ>::ld(Q1, (int64_t)j * N + i);
    CT q1 = Elem<TQ>::ld(Q1, (int64_t)(j + 1) * N + i);
    CT q2 = Elem<TQ>::ld(Q1, (int64_t)(j + 2) * N + i);
    CT q3 = Elem<TQ>::ld(Q1, (int64_t)(j + 3) * N + i);
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      acc[c] = fma(q0, sY[(j + 0) * CB + c], acc[c]);
      acc[c] = fma(q1, sY[(j + 1) * CB + c], acc[c]);
      acc[c] = fma(q2, sY[(j + 2) * CB + c], acc[c]);
      acc[c] = fma(q3, sY[(j + 3) * CB + c], acc[c]);
    }
  }
  for (; j < mq; ++j) {
    CT q = Elem<TQ>::ld(Q1, (int64_t)j * N + i);
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[c] = fma(q, sY[j * CB + c], acc[c]);
  }
  if (Qlo != nullptr)
    for (int jl = 0; jl < pm; ++jl) {   // remainder of column jl + 1: Y row jl + 1 (sY row jl)
      CT q = Elem<TQ>::ld(Qlo, (int64_t)jl * N + i);
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[c] = fma(q, sY[jl * CB + c], acc[c]);
    }
  const int ml = map[i];
  const CT sc = normalized ? (CT)dinv[i] : CT(1);
  const bool live = !normalized || sc > CT(0);
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    int lab = lab0 + c;
    if (lab >= C) break;
    CT v = ml ? (ml - 1 == lab ? CT(1) : CT(0)) : sc * acc[c] + (live ? sK[c] : CT(0));
    U[(int64_t)lab * N + i] = (TU)v;
  }
}

template <typename TQ, typename TU>
static int reconstruct_t(const Graph* g, const void* Q, const uint16_t* Qlo, int m, const double* Y, int C,
                         const uint8_t* map, void* U, hipStream_t s) {
  using CT = typename Elem<TQ>::C;
  const TQ* lo = reinterpret_cast<const TQ*>(Qlo);   // non-null only with TQ = uint16_t
  const int pm = std::min(kPairCols, m - 1);
  for (int lab0 = 0; lab0 < C; lab0 += 8) {
    int rem = C - lab0;
    if (rem <= 4) {
      size_t sh = (size_t)m * 4 * sizeof(CT);
      k_reconstruct<TQ, TU, 4><<<nblocks(g->N, 256), 256, sh, s>>>((const TQ*)Q, lo, pm, g->N, m, Y, C, lab0, map,
                                                                    (const TU*)g->dinv, g->normalized, (TU*)U);
    } else {
      size_t sh = (size_t)m * 8 * sizeof(CT);
      k_reconstruct<TQ, TU, 8><<<nblocks(g->N, 256), 256, sh, s>>>((const TQ*)Q, lo, pm, g->N, m, Y, C, lab0, map,
                                                                    (const TU*)g->dinv, g->normalized, (TU*)U);
    }
    RW_LAUNCH_CHECK();
  }
  return RW_OK;
}

static int reconstruct(const Graph* g, const void* Q, int qdt, int m, const double* Y, int C, const uint8_t* map,
                       void* U, hipStream_t s) {
  const BasisView b = basis_view(g->N, Q, qdt);
  if (b.dt == RW_BF16 && C <= 8) return reconstruct_mfma(g, b.hi, b.lo, m, Y, C, map, U, s);
  RW_CHECK((size_t)m * 8 * 8 <= 65536, RW_EINVAL, "m = %d too large for the reconstruction tile", m);
  if (g->dtype == RW_F64) {
    if (b.dt == RW_F64) return reconstruct_t<double, double>(g, b.hi, nullptr, m, Y, C, map, U, s);
    if (b.dt == RW_F32) return reconstruct_t<float, double>(g, b.hi, nullptr, m, Y, C, map, U, s);
    return reconstruct_t<uint16_t, double>(g, b.hi, b.lo, m, Y, C, map, U, s);
  }
  if (b.dt == RW_F64) return reconstruct_t<double, float>(g, b.hi, nullptr, m, Y, C, map, U, s);
  if (b.dt == RW_F32) return reconstruct_t<float, float>(g, b.hi, nullptr, m, Y, C, map, U, s);
  return reconstruct_t<uint16_t, float>(g, b.hi, b.lo, m, Y, C, map, U, s);
}

int reconstruct_any(const Graph* g, const void* Q, int qdt, int m, const double* Y, int C, const uint8_t* map,
                    void* U, hipStream_t s) {
  return reconstruct(g, Q, qdt, m, Y, C, map, U, s);
}

// ---------------------------------------------------------------------------------------------
// Choice of m (Sec. III-A1): f_k(m) = min_{||a|| <= rho} ||Q_s[:, :m] a - b_k||^2.
// Per candidate m, with ms = min(S, m): for m <= S the m x m normal matrix G = Q_s^T Q_s (leading
// block) and g_k = Q_s^T b_k; for m > S the S x S matrix P = Q_s Q_s^T over the first m columns and
// b_k.  One eigendecomposition per candidate (shared by the labels, right-hand sides rotated along)
// turns the constrained problem into the secular equation ||a(mu)|| = rho in mu >= 0:
//   m <= S:  ||a||^2 = sum g_i^2 / (w_i + mu)^2,     f = ||b||^2 - sum g_i^2 (w_i + 2 mu) / (w_i + mu)^2
//   m >  S:  ||a||^2 = sum b_i^2 w_i / (w_i + mu)^2, f = sum b_i^2 mu^2 / (w_i + mu)^2
// with (w_i) the eigenvalues and (g_i), (b_i) the rotated right-hand sides.  mu = 0 when the
// minimum-norm least-squares fit is feasible, else bisection (geometric) to relative 1e-15.
// Candidate matrices are zero-padded to a common size; padding adds w = 0 with zero right-hand side.
// ---------------------------------------------------------------------------------------------
__global__ void k_fit_build(const int* cand, int64_t S, int ma, int C, int ms, const double* Qs, const double* Gq,
                            const double* Gb, const double* Us, double* A, double* R) {
  const int ci = blockIdx.x;
  const int m = cand[ci];
  double* Ab = A + (int64_t)ci * ms * ms;
  double* Rb = R + (int64_t)ci * ms * C;
  if (m <= S) {
    for (int64_t t = threadIdx.x; t < (int64_t)ms * ms; t += blockDim.x) {
      int i = (int)(t % ms), j = (int)(t / ms);
      Ab[t] = (i < m && j < m) ? Gq[i + (int64_t)j * ma] : 0.0;
    }
    for (int64_t t = threadIdx.x; t < (int64_t)ms * C; t += blockDim.x) {
      int i = (int)(t % ms), k = (int)(t / ms);
      Rb[t] = i < m ? Gb[i + (int64_t)k * ma] : 0.0;
    }
  } else {   // ms == S
    for (int64_t t = threadIdx.x; t < (int64_t)ms * ms; t += blockDim.x) {
      int i = (int)(t % ms), j = (int)(t / ms);
      double acc = 0.0;
      for (int c = 0; c < m; ++c) acc += Qs[i + (int64_t)c * S] * Qs[j + (int64_t)c * S];
      Ab[t] = acc;
    }
    for (int64_t t = threadIdx.x; t < (int64_t)ms * C; t += blockDim.x) {
      int i = (int)(t % ms), k = (int)(t / ms);
      Rb[t] = Us[i + (int64_t)k * S];
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) { return wave_sum64(v); }

// rho of eq. (24): sqrt(1^T D 1) from the graph's device sum for the normalized operator, else sqrt(N)
__device__ __forceinline__ double fit_rho(const double* sums, double n_nodes) {
  return sqrt(sums != nullptr ? sums[0] : n_nodes);
}

// one wave per (candidate, label); lane-parallel sums reduced by butterflies, so all lanes agree
__global__ __launch_bounds__(64) void k_fit_secular(const int* cand, int ncand, int64_t S, int C, int ms,
                                                    const double* W, const double* R, const double* Us,
                                                    const double* sums, double n_nodes, double* fvals) {
  const double rho = fit_rho(sums, n_nodes);
  const int ci = blockIdx.x, k = blockIdx.y;
  const int lane = threadIdx.x;
  const int m = cand[ci];
  const bool small_m = m <= S;
  const double* w = W + (int64_t)ci * ms;
  const double* g = R + (int64_t)ci * ms * C + (int64_t)k * ms;
  double bn = 0.0;
  for (int64_t i = lane; i < S; i += 64) bn += Us[i + (int64_t)k * S] * Us[i + (int64_t)k * S];
  const double bnorm2 = wave_sum(bn);
  const double rho2 = rho * rho;
  // this lane's g_i^2 and w_i (i = lane + 64 q), held in registers across the bisection
  constexpr int kQ = 16;   // ms <= 1024
  const int nq = (ms + 63) / 64;
  double g2v[kQ], wv[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int i = lane + 64 * q;
    const bool in = q < nq && i < ms;
    const double gi = in ? g[i] : 0.0;
    g2v[q] = gi * gi;
    wv[q] = in ? w[i] : 0.0;
  }
  auto norm2 = [&](double mu) -> double {
    double acc = 0.0;
    int inf = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      if (q >= nq) break;   // uniform
      const double gi2 = g2v[q];
      if (gi2 == 0.0) continue;
      const double wi = fmax(wv[q], 0.0), den = wi + mu;
      if (den <= 0.0) { inf = 1; continue; }
      acc += small_m ? gi2 / (den * den) : gi2 * wi / (den * den);
    }
    double tot = wave_sum(acc);
    double anyinf = wave_sum((double)inf);
    return anyinf > 0.0 ? (double)INFINITY : tot;
  };
  auto fval = [&](double mu) -> double {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      if (q >= nq) break;   // uniform
      const double gi2 = g2v[q];
      if (gi2 == 0.0) continue;
      const double wi = fmax(wv[q], 0.0), den = wi + mu;
      if (small_m) acc += gi2 * (wi + 2.0 * mu) / (den * den);
      else acc += den > 0.0 ? gi2 * (mu / den) * (mu / den) : gi2;
    }
    double tot = wave_sum(acc);
    return small_m ? fmax(bnorm2 - tot, 0.0) : tot;
  };
  double mu = 0.0;
  if (!(norm2(0.0) <= rho2)) {
    double gn = 0.0, wm = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      if (q >= nq) break;   // uniform
      const int i = lane + 64 * q;
      if (i < ms) {
        gn += g2v[q];
        wm = fmax(wm, wv[q]);
      }
    }
    gn = wave_sum(gn);
    wm = wave_max64(wm);
    double hi = small_m ? sqrt(gn) / rho : sqrt(fmax(wm, 1e-300) * gn) / rho;
    hi = fmax(hi, 1e-300);
    while (norm2(hi) > rho2) hi *= 2.0;
    double lo = 0.0;
    for (int it = 0; it < 400 && hi - lo > 1e-15 * hi; ++it) {
      double mid = lo > 0.0 ? sqrt(lo * hi) : 0.5 * hi;
      if (mid <= lo || mid >= hi) mid = 0.5 * (lo + hi);
      if (norm2(mid) > rho2) lo = mid;
      else hi = mid;
    }
    mu = hi;
  }
  const double f = fval(mu);
  if (lane == 0) fvals[ci + (int64_t)k * ncand] = f;
}

// Screening of the choice of m by one Cholesky factorization.  The leading m x m block of
// G = Q_s^T Q_s is factorized by the leading block of G's lower Cholesky factor L, so one
// factorization gives, for every m at once, the unconstrained least-squares fit of each label:
//   z = L^{-1} g,  r(m) = ||b||^2 - sum_{j<m} z_j^2,  a(m) = L_m^{-T} z_m.
// r(m) <= f(m) (the constraint can only raise the minimum), so r(m) > f_max decides "fails"; when the
// fit is also feasible (||a(m)|| <= rho) it solves the constrained problem, f(m) = r(m), which decides
// "passes" or "fails" outright.  Rounding: the factorization is exact for G + E with
// ||E|| <= c (m^2 + S) u trace(G_m) (Gram sums and factorization), which moves r(m) by a^T E a to
// first order, so each decision keeps a band of 16 (m^2 + S) u trace(G_m) ||a(m)||^2 (plus 1e-10
// relative) around f_max.  Everything else (an active or
// nearly active constraint, a value inside the band, or m beyond the first pivot below 1e-12 of its
// diagonal entry, where G's leading block is numerically singular, as for every m > S) is left to
// the eigen-based evaluation.  The factorization stops at the first m whose residual is at most f_max
// for every label; larger m stay undecided (the search never needs them unless that m is undecided).
// One workgroup; everything lives in LDS, which bounds the factorized size to KM columns (m > KM stays
// undecided).  The factorization is right-looking with unscaled columns (Schur complements
// A(i,j) -= A(i,k) A(j,k) / A(k,k)), one barrier per column; the right-hand sides are updated alongside
// (z_k = g_k / sqrt(A(k,k))), and the stopping test for k reads the residuals left by column k - 1.
// Then Ri = L^{-T} column by column (one wave per column, back substitution in axpy form with the
// solved entry broadcast from its lane), and per label the row prefix sums P.
__device__ __forceinline__ int scr_lo(int i, int j, int KM) { return j * KM - ((j * (j - 1)) >> 1) + (i - j); }  // i >= j
__device__ __forceinline__ int scr_up(int i, int j) { return ((j * (j + 1)) >> 1) + i; }                        // i <= j

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int kScreenMaxKM = 192;   // the inverse's forward substitution: 3 row slots x 12 column slots

static size_t screen_lds_bytes(int KM, int C) {
  return ((size_t)KM * (KM + 1) + 2 * (size_t)KM * C + 2 * (size_t)KM + 3 * (size_t)C) * sizeof(double);
}

static int screen_cols(int ma, int C) {
  int KM = std::min(ma, kScreenMaxKM);
  while (KM > 0 && screen_lds_bytes(KM, C) > kLdsLimit) --KM;
  return KM;
}

__global__ __launch_bounds__(1024) void k_fit_screen(int ma, int KM, int C, int64_t S, const double* Gq,
                                                     const double* Gb, const double* Us, const double* sums,
                                                     double n_nodes, double f_max, double* F, int* cls) {
  const double rho = fit_rho(sums, n_nodes), rho2 = rho * rho;
  extern __shared__ double sm[];
  const int tri = KM * (KM + 1) / 2;
  double* A = sm;              // packed lower (column-major): G_m, then L column by column; later Ri (packed upper)
  double* B = A + tri;         // packed upper: the prefix sums P
  double* G = B + tri;         // KM x C right-hand sides g = Q_s^T u, updated
  double* Z = G + KM * C;      // KM x C, z = L^{-1} g
  double* rd = Z + KM * C;     // 1 / L(k, k)
  double* sr = rd + KM;        // 2 x C running residuals (alternating by column parity)
  double* sbn = sr + 2 * C;    // ||b||^2 per label
  double* gd = sbn + C;        // diagonal of G_m (the pivot test and the error bound read it)
  __shared__ int s_kf;
  const int tid = threadIdx.x;
  if (tid < 64) {
    for (int c = 0; c < C; ++c) {
      double acc = 0.0;
      for (int64_t i = tid; i < S; i += 64) acc += Us[i + c * S] * Us[i + c * S];
      acc = wave_sum64(acc);
      if (tid == 0) {
        sbn[c] = acc;
        sr[c] = acc;
      }
    }
  }
  for (int t = tid; t < KM * KM; t += blockDim.x) {
    const int i = t % KM, j = t / KM;
    if (i >= j) A[scr_lo(i, j, KM)] = Gq[i + (int64_t)j * ma];
  }
  for (int t = tid; t < KM * C; t += blockDim.x) G[t] = Gb[t % KM + (int64_t)(t / KM) * ma];
  for (int t = tid; t < KM; t += blockDim.x) gd[t] = Gq[t + (int64_t)t * ma];
  if (tid == 0) s_kf = KM;
  __syncthreads();
  // Cholesky with early stop, left-looking (column k of L is formed from the earlier columns only when its
  // step comes): stop at the first small pivot (numerically singular leading block) or as soon as every
  // label's residual r(k) is at most f_max (no larger m is needed: the first m that can pass is at most k)
  // Columns go in pairs (k, k+1): one pass forms both Schur columns from the same rows of L (the
  // L(i, k) L(k+1, k) term of column k+1 is applied once column k is final), and the decisions for k+1
  // are taken by every thread from values no thread changes in that phase, so a pair costs two barriers.
  // sr holds the residuals before the pair (buffer (k / 2) & 1) and after it (the other buffer).
  // L(k+1, k) is read by every thread in the pair's second phase, so it is stored after that phase's
  // barrier (pend_k, pend_l: the same in every thread).
  int pend_k = -1;
  double pend_l = 0.0;
  for (int k = 0; k < KM; k += 2) {
    const double* srk = sr + ((k >> 1) & 1) * C;
    double* srn = sr + (((k >> 1) + 1) & 1) * C;
    if (pend_k >= 0 && tid == 0) A[scr_lo(pend_k + 1, pend_k, KM)] = pend_l;   // no reader until after the loop
    pend_k = -1;
    if (k > 0) {
      double worst = 0.0;
      for (int c = 0; c < C; ++c) worst = fmax(worst, srk[c]);
      if (worst <= f_max) {   // uniform
        if (tid == 0) s_kf = k;
        break;
      }
    }
    const bool two = k + 1 < KM;
    {   // Schur columns c_i = A(i, k) - sum_{j<k} L(i, j) L(k, j) (rows i >= k) and the same for k + 1
        // without its j = k term (rows i >= k + 1): one quad of lanes per row
      const int r = tid >> 2, sub = tid & 3, i = k + r;
      double acc0 = 0.0, acc1 = 0.0;
      if (i < KM) {
        for (int j = sub; j < k; j += 4) {
          const double lij = A[scr_lo(i, j, KM)];
          acc0 += lij * A[scr_lo(k, j, KM)];
          if (two) acc1 += lij * A[scr_lo(k + 1, j, KM)];
        }
      }
      acc0 = quad_sum(acc0);
      acc1 = quad_sum(acc1);
      if (sub == 0 && i < KM) {
        A[scr_lo(i, k, KM)] -= acc0;
        if (two && i > k) A[scr_lo(i, k + 1, KM)] -= acc1;
      }
    }
    lds_barrier();
    const double dkk = A[scr_lo(k, k, KM)];
    if (!(dkk > 1e-12 * gd[k]) || !isfinite(dkk)) {   // uniform
      if (tid == 0) s_kf = k;
      break;
    }
    const double lkk = sqrt(dkk), rk = 1.0 / lkk;
    if (tid < C) Z[k + tid * KM] = G[k + tid * KM] / lkk;
    if (tid == 0) rd[k] = rk;
    // column k + 1: stop before it when every residual after column k is small enough, or at a small pivot
    bool stop1 = !two;
    double Lk1 = 0.0, l1 = 1.0, r1 = 1.0;
    if (two) {
      double worst = 0.0;
      for (int c = 0; c < C; ++c) {
        const double z = G[k + c * KM] / lkk;
        worst = fmax(worst, srk[c] - z * z);
      }
      Lk1 = A[scr_lo(k + 1, k, KM)] * rk;
      const double dk1 = A[scr_lo(k + 1, k + 1, KM)] - Lk1 * Lk1;
      stop1 = worst <= f_max || !(dk1 > 1e-12 * gd[k + 1]) || !isfinite(dk1);   // uniform
      if (!stop1) {
        l1 = sqrt(dk1);
        r1 = 1.0 / l1;
      }
    }
    if (stop1) {   // finish column k only
      for (int i = k + 2 + tid; i < KM; i += blockDim.x) {
        const double l = A[scr_lo(i, k, KM)] * rk;
        A[scr_lo(i, k, KM)] = l;
      }
      if (two) {
        pend_k = k;
        pend_l = Lk1;
      }
      if (tid < C) {
        const double z = G[k + tid * KM] / lkk;
        srn[tid] = srk[tid] - z * z;
      }
      if (tid == 0) s_kf = two ? k + 1 : KM;
      break;
    }
    // z_{k+1} from g_{k+1} after column k, and the residuals after the pair
    if (tid < C) {
      const double z0 = G[k + tid * KM] / lkk;
      const double z1 = (G[k + 1 + tid * KM] - Lk1 * (G[k + tid * KM] * rk)) / l1;
      Z[k + 1 + tid * KM] = z1;
      srn[tid] = (srk[tid] - z0 * z0) - z1 * z1;
    }
    if (tid == 0) rd[k + 1] = r1;
    pend_k = k;
    pend_l = Lk1;
    // rows below the pair: L(i, k), L(i, k+1) and the right-hand sides
    for (int i = k + 2 + tid; i < KM; i += blockDim.x) {
      const double l0 = A[scr_lo(i, k, KM)] * rk;
      const double l1i = (A[scr_lo(i, k + 1, KM)] - l0 * Lk1) * r1;
      A[scr_lo(i, k, KM)] = l0;
      A[scr_lo(i, k + 1, KM)] = l1i;
      for (int c = 0; c < C; ++c) {
        const double gk = G[k + c * KM] * rk;
        const double gk1 = (G[k + 1 + c * KM] - Lk1 * gk) * r1;
        G[i + c * KM] -= l0 * gk + l1i * gk1;
      }
    }
    lds_barrier();
  }
  __syncthreads();
  if (pend_k >= 0 && tid == 0) A[scr_lo(pend_k + 1, pend_k, KM)] = pend_l;
  __syncthreads();
  const int kf = s_kf;      // leading blocks of size <= kf are factorized
  // Ri = L^{-T} (packed upper, over A): with D = diag(L) and the unit lower M = L D^{-1} (M(i, k) = L(i, k)
  // rd[k]), L^{-1} = D^{-1} M^{-1}.  Y = M^{-1} by forward substitution on all columns at once, thread
  // (lane, wave) holding Y(i, j) for the rows i = lane + 64 s and the columns j = wave + 16 t (each wave its
  // own columns: no barriers; step k = 16 T + w with T unrolled, so that row k's slot is known at compile
  // time); then Ri(j, i) = Y(i, j) rd[i], written over L once every wave has read it
  {
    constexpr int YR = (kScreenMaxKM + 63) / 64, YC = (kScreenMaxKM + 15) / 16;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double y[YR][YC];
#pragma unroll
    for (int s = 0; s < YR; ++s)
#pragma unroll
      for (int t = 0; t < YC; ++t) y[s][t] = (lane + 64 * s == wave + 16 * t && lane + 64 * s < kf) ? 1.0 : 0.0;
    static_for<0, YC>([&](auto Tc) {
      constexpr int T = decltype(Tc)::value, SK = T / 4;   // row slot of k = 16 T + w
      for (int w = 0; w < 16; ++w) {
        const int k = 16 * T + w;
        if (k >= kf - 1) return;   // uniform
        const double rk = rd[k];
        double l[YR];
#pragma unroll
        for (int s = 0; s < YR; ++s) {
          const int i = lane + 64 * s;
          const double v = A[scr_lo(min(max(i, k + 1), kf - 1), k, KM)];
          l[s] = (i > k && i < kf) ? v * rk : 0.0;
        }
        static_for<0, T + 1>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          const double yk = lane_read(y[SK][t], k & 63);
#pragma unroll
          for (int s = 0; s < YR; ++s) {
            y[s][t] -= l[s] * yk;
            asm volatile("" : "+v"(y[s][t]));   // updated here, not sunk to later uses
          }
        });
      }
    });
    __syncthreads();   // every wave has read L
#pragma unroll
    for (int s = 0; s < YR; ++s)
#pragma unroll
      for (int t = 0; t < YC; ++t) {
        const int i = lane + 64 * s, j = wave + 16 * t;
        if (i < kf && j <= i) A[scr_up(j, i)] = y[s][t] * rd[i];
      }
  }
  __syncthreads();
  // per m in [1, ma]: residual r(m) = ||b||^2 - sum_{j<m} z_j^2 and the fit's squared norm
  // ||a(m)||^2 = sum_{i<m} P(i, m-1)^2 with the row prefix sums P(i, j) = sum_{i<=j'<=j} Ri(i, j') z_j'
  double bmax = 0.0;
  for (int c = 0; c < C; ++c) bmax = fmax(bmax, sbn[c]);
  const double band0 = 1e-10 * (f_max + bmax);
  // per-thread state for m = 1 + tid (ma <= 1024)
  const int m = 1 + tid;
  double trg = 0.0;
  if (m <= kf)
    for (int k = 0; k < m; ++k) trg += gd[k];
  // Gram rounding (S terms per entry) plus the factorization's (m^2): ||E|| <= 16 (m^2 + S) u trace(G_m)
  const double ebound = 16.0 * ((double)m * (double)m + (double)S) * 1.1102230246251565e-16 * trg;
  double rmax = 0.0;
  bool anyfail = false, allpass = true;
  for (int c = 0; c < C; ++c) {
    const double* z = Z + c * KM;
    if (tid < kf) {
      const int i = tid;
      double acc = 0.0;
      for (int j = i; j < kf; ++j) {
        acc += A[scr_up(i, j)] * z[j];
        B[scr_up(i, j)] = acc;
      }
    }
    __syncthreads();
    if (m <= kf) {
      double zz = 0.0, an = 0.0;
      for (int j = 0; j < m; ++j) zz += z[j] * z[j];
      for (int i = 0; i < m; ++i) {
        const double v = B[scr_up(i, m - 1)];
        an += v * v;
      }
      const double r = fmax(sbn[c] - zz, 0.0);
      rmax = fmax(rmax, r);
      const double band = band0 + ebound * an;
      if (r > f_max + band) anyfail = true;
      if (!(r < f_max - band) || !(an <= 0.99 * rho2)) allpass = false;
    }
    __syncthreads();
  }
  if (m <= ma) {
    int cl = 2;
    if (m <= kf) {
      if (anyfail) cl = 0;
      else if (allpass) cl = 1;
    }
    F[m] = m <= kf ? rmax : 0.0;
    cls[m] = cl;
  }
  if (tid == 0) {
    cls[0] = kf;
    F[0] = 0.0;
  }
}

// ---------------------------------------------------------------------------------------------

// the seed rows of the first ma stored columns (hi + lo for the pair form), B Q_n, U_hat_s, op_ss U_hat_s
static int seed_gather(const Graph* g, const void* Q, int qdt, int ma, const SolveWork& w, int64_t S, int C,
                       hipStream_t s) {
  const GridDev G = grid_of(g);
  const BasisView b = basis_view(g->N, Q, qdt);
#define RW_GATHER(TQ, LO)                                                                                   \
  k_seed_gather<TQ><<<(unsigned)S, 256, 0, s>>>(G, g->normalized, (const TQ*)b.hi, LO, ma, w.seeds, w.map,       \
                                                g->weight, g->degree, g->sums, S, C, w.Qs, w.GB, w.Hs, w.Us, w.gs, \
                                                w.Bg)
  if (b.dt == RW_F64) RW_GATHER(double, nullptr);
  else if (b.dt == RW_F32) RW_GATHER(float, nullptr);
  else RW_GATHER(uint16_t, b.lo);
#undef RW_GATHER
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// Validates, sorts and de-duplicates the seeds into caller buffers (v: S pairs of scratch; nodes, labels:
// S entries); *S_out receives the number of distinct seeds.  Allocates nothing.
static int host_seeds_into(const Graph* g, const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C,
                           std::pair<int64_t, int32_t>* v, int64_t* nodes, int32_t* labels, int64_t* S_out) {
  RW_CHECK(S >= 1, RW_EINVAL, "at least one seed is required");
  RW_CHECK(seed_node != nullptr && seed_label != nullptr, RW_EINVAL, "null seed arrays");
  RW_CHECK(C >= 1 && C <= 255, RW_EINVAL, "C must be in [1, 255] (got %d)", C);
  for (int64_t k = 0; k < S; ++k) {
    RW_CHECK(seed_node[k] >= 0 && seed_node[k] < g->N, RW_EINVAL, "seed %lld: node %lld out of range",
             (long long)k, (long long)seed_node[k]);
    RW_CHECK(seed_label[k] >= 0 && seed_label[k] < C, RW_EINVAL, "seed %lld: label %d out of range",
             (long long)k, seed_label[k]);
    v[k] = {seed_node[k], seed_label[k]};
  }
  std::sort(v, v + S);
  int64_t n = 0;
  for (int64_t k = 0; k < S; ++k) {
    if (k > 0 && v[k].first == v[k - 1].first) {
      RW_CHECK(v[k].second == v[k - 1].second, RW_EINVAL, "node %lld seeded with labels %d and %d",
               (long long)v[k].first, v[k - 1].second, v[k].second);
      continue;
    }
    nodes[n] = v[k].first;
    labels[n] = v[k].second;
    ++n;
  }
  *S_out = n;
  return RW_OK;
}

// Host bytes that hold the status words read back at the end of a solve.
constexpr size_t kStatusStageBytes = 512;

// The solve on sorted, distinct seeds (S of them; the workspace is laid out for S_cap >= S).  final_stage:
// host memory (kStatusStageBytes) for the three status words read at the end (pinned staging when null).
static int solve_impl(rw_graph h, const void* Q, int q_dtype, const double* lambda, int m_avail, const int64_t* nodes,
                      const int32_t* labels, int64_t S, int64_t S_cap, int C, double eps, void* U, const SolveWork& w,
                      hipStream_t stream, rw_solve_info* info, void* final_stage) {
  const Graph* g = &h->g;
  // seeds to the device; map of seeded nodes
  RW_HIP(hipMemcpyAsync(w.seeds, nodes, S * sizeof(int64_t), hipMemcpyHostToDevice, stream));
  RW_HIP(hipMemcpyAsync(w.labels, labels, S * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  // the anchoring check is queued here and read with the pivot test at the end
  const int* unanchored = nullptr;
  RW_TRY(anchor_launch(&h->g, w.seeds, S, w.anc, stream, &unanchored));
  k_clear_map<<<nblocks(g->N, 256), 256, 0, stream>>>(w.map, g->N);
  RW_LAUNCH_CHECK();
  k_set_map<<<nblocks(S, 256), 256, 0, stream>>>(w.map, w.seeds, w.labels, S);
  RW_LAUNCH_CHECK();
  const int ma = m_avail;
  RW_TRY(seed_gather(g, Q, q_dtype, ma, w, S, C, stream));
  RW_HIP(hipMemsetAsync(w.nbad, 0, sizeof(int), stream));
  // choice of m (on the stored columns)
  int m = ma;
  int probes = 0;
  double f_max = 0.0, f_worst = 0.0;
  if (eps > 0.0) {
    f_max = (double)S * eps * eps;
    RW_TRY(gram(RW_F64, w.Qs, S, w.Qs, S, S, ma, ma, w.Gq, w.partial, stream, true));
    RW_TRY(gram(RW_F64, w.Qs, S, w.Us, S, S, ma, C, w.Gb, w.partial, stream));
    // rho (eq. (24)) is formed on the device from the graph's degree sum
    const double* rho_sums = g->normalized ? g->sums : nullptr;
    // search: lo = largest m known to fail (1 = none), hi = smallest m known to pass (ma + 1 = none)
    int lo = 1, hi = ma + 1;
    std::vector<std::pair<int, double>> evaluated;
    const int KM = (C <= 64 && ma <= 1024) ? screen_cols(ma, C) : 0;   // one thread per m in the classification
    const bool screened = KM >= 1;
    if (screened) {
      static bool attr = false;
      if (!attr) {
        RW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_fit_screen),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
        attr = true;
      }
      k_fit_screen<<<1, 1024, screen_lds_bytes(KM, C), stream>>>(ma, KM, C, S, w.Gq, w.Gb, w.Us, rho_sums,
                                                                  (double)g->N, f_max, w.scrF, w.scrCls);
      RW_LAUNCH_CHECK();
      // F and the classes are adjacent in the workspace: one copy of the span that holds both
      const size_t cls_off = reinterpret_cast<const char*>(w.scrCls) - reinterpret_cast<const char*>(w.scrF);
      const size_t span = cls_off + (size_t)(ma + 1) * sizeof(int);
      void* stage = nullptr;
      RW_TRY(host_stage(span, &stage));
      const double* frs = static_cast<const double*>(stage);
      const int* clss = reinterpret_cast<const int*>(static_cast<const char*>(stage) + cls_off);
      RW_HIP(hipMemcpyAsync(stage, w.scrF, span, hipMemcpyDeviceToHost, stream));
      RW_HIP(hipStreamSynchronize(stream));
      const std::vector<int> cls(clss, clss + ma + 1);
      const std::vector<double> fr(frs, frs + ma + 1);
      // f is non-increasing in m: the first m not known to fail bounds lo, the first known pass bounds hi
      int m0 = 2;
      while (m0 <= ma && cls[m0] == 0) ++m0;
      lo = std::min(m0, ma) - 1;    // when every m fails, m_avail is still evaluated for its fit value
      for (int m = m0; m <= ma; ++m)
        if (cls[m] == 1) {
          hi = m;
          evaluated.push_back({m, fr[m]});
          break;
        }
    }
    const int maxc = fit_cands(ma);
    std::vector<double> fh((size_t)maxc * C);
    std::vector<int> cand;
    // candidate list lives in the first maxc ints of the K buffer (unused until the final solve)
    int* cand_buf = reinterpret_cast<int*>(w.K);
    const int msmax = (int)std::min<int64_t>(S, ma);
    RW_CHECK(msmax <= 1022, RW_EINVAL, "choice of m supports min(S, m_avail) <= 1022");
    while (hi - lo > 1) {
      ++probes;
      cand.clear();
      int span = hi - lo - 1;
      if (screened) {
        // the screen leaves lo + 1 undecided and usually passes a few m later: the next 8 m in order on the
        // first probe (the batch's cost grows with its largest candidate), the next 32 on later ones
        const int take = probes == 1 ? 8 : 32;
        for (int mm = std::max(lo + 1, 2); mm < hi && (int)cand.size() < std::min(take, maxc); ++mm) cand.push_back(mm);
      } else {
        int nc = std::min(span, maxc);
        for (int q = 1; q <= nc; ++q) {
          int mm = lo + (int)(((int64_t)span * q + nc - 1) / nc);
          if (mm < 2) mm = 2;
          if (cand.empty() || mm > cand.back()) cand.push_back(mm);
        }
      }
      int ncand = (int)cand.size();
      RW_HIP(hipMemcpyAsync(cand_buf, cand.data(), ncand * sizeof(int), hipMemcpyHostToDevice, stream));
      // candidate problems are padded to the largest candidate's size (S once a candidate exceeds S)
      const int msp = (int)std::min<int64_t>(S, cand.back());
      k_fit_build<<<ncand, 256, 0, stream>>>(cand_buf, S, ma, C, msp, w.Qs, w.Gq, w.Gb, w.Us, w.fitA, w.fitR);
      RW_LAUNCH_CHECK();
      // eigenvalues and rotated right-hand sides through the tridiagonal form (each candidate at its own
      // order), the Jacobi solver when eigenvalues cluster or the batch does not fit
      int est = RW_ENOCONV;
      const double* tri_flag = nullptr;   // the tridiagonal path's cluster flag, read with the fit values
      if (ncand <= kTriBatchMax && tridiag_batch_fits(msp)) {
        int sizes[kTriBatchMax];
        bool ok = true;
        for (int q = 0; q < ncand; ++q) {
          sizes[q] = (int)std::min<int64_t>(S, cand[q]);
          ok = ok && tridiag_batch_fits(sizes[q]);
        }
        if (ok) {
          RW_TRY(syev_tridiag_rhs(w.fitA, msp, sizes, ncand, w.fitR, C, w.fitW, w.fitWork, w.fitWorkCount, stream,
                                  &tri_flag));
          est = RW_OK;
        }
      }
      // fit values (eq. (24)) from the eigenpairs; when the tridiagonal path flags clustered eigenvalues (it then
      // leaves fitW and fitR as they were) they are discarded and formed again after the Jacobi solver
      for (int pass = 0; pass < 2; ++pass) {
        if (est == RW_ENOCONV)
          RW_TRY(syev_batched(w.fitA, w.fitW, nullptr, w.fitR, C, msp, ncand, w.fitWork, stream));
        k_fit_secular<<<dim3(ncand, C), 64, 0, stream>>>(cand_buf, ncand, S, C, msp, w.fitW, w.fitR, w.Us,
                                                          rho_sums, (double)g->N, w.fvals);
        RW_LAUNCH_CHECK();
        void* stage = nullptr;
        RW_TRY(host_stage(((size_t)ncand * C + 1) * sizeof(double), &stage));
        double* hs = static_cast<double*>(stage);
        hs[(size_t)ncand * C] = 0.0;
        RW_HIP(hipMemcpyAsync(hs, w.fvals, (size_t)ncand * C * sizeof(double), hipMemcpyDeviceToHost, stream));
        if (est == RW_OK)
          RW_HIP(hipMemcpyAsync(hs + (size_t)ncand * C, tri_flag, sizeof(double), hipMemcpyDeviceToHost, stream));
        RW_HIP(hipStreamSynchronize(stream));
        std::copy(hs, hs + (size_t)ncand * C, fh.begin());
        const double fl = hs[(size_t)ncand * C];
        if (est == RW_ENOCONV || fl == 0.0) break;
        est = RW_ENOCONV;
      }
      int first_pass = -1;
      for (int q = 0; q < ncand; ++q) {
        double worst = 0.0;
        for (int c = 0; c < C; ++c) worst = std::max(worst, fh[(size_t)c * ncand + q]);
        evaluated.push_back({cand[q], worst});
        if (first_pass < 0 && worst <= f_max) first_pass = q;
      }
      if (first_pass < 0) {
        lo = cand.back();
      } else {
        hi = cand[first_pass];
        if (first_pass > 0) lo = cand[first_pass - 1];
      }
    }
    m = hi <= ma ? hi : ma;
    f_worst = INFINITY;
    for (auto& e : evaluated)
      if (e.first == m) f_worst = e.second;
  }
  // the FP64 basis of the first m columns: c_j, n_j by one pass over Q, then the seed rows in place
  RW_TRY(null_stats(g, Q, q_dtype, m, w.npart, w.cn, w.nbad, stream));
  k_seed_correct<<<nblocks(S * m, 256), 256, 0, stream>>>(w.Qs, w.GB, w.gs, w.Bg, w.cn, S, m);
  RW_LAUNCH_CHECK();
  // reduced system K = Lambda - Q'_s^T (B Q'_n), Y = Q'_s^T (op_ss U_hat_s), and its solve (the batched solve
  // forms and solves each image's system with the same code)
  k_reduced<<<reduced_grid(m, C), 256, 0, stream>>>(m, C, S, w.Qs, w.GB, w.Hs, lambda, 0.0, w.K,
                                                                     w.Y);
  RW_LAUNCH_CHECK();
  RW_TRY(lu_solve(w.K, m, w.Y, C, w.stat, stream));
  RW_TRY(solve_coeffs(w.Y, m, C, w.cn, g, stream));
  // the reconstruction is queued before the pivot test is read (one wait for both); U is not valid when
  // the test fails
  RW_TRY(reconstruct(g, Q, q_dtype, m, w.Y, C, w.map, U, stream));
  // stat and the null-column flag are adjacent in the workspace (one copy); the anchor flag follows them
  const size_t nbad_off = reinterpret_cast<const char*>(w.nbad) - reinterpret_cast<const char*>(w.stat);
  const size_t bad_off = (nbad_off + sizeof(int) + 7) & ~size_t(7);
  RW_CHECK(bad_off + sizeof(int) <= kStatusStageBytes, RW_EINVAL, "status staging too small (%zu bytes)", bad_off);
  void* stage = final_stage;
  if (stage == nullptr) RW_TRY(host_stage(kStatusStageBytes, &stage));
  char* hs = static_cast<char*>(stage);
  RW_HIP(hipMemcpyAsync(hs, w.stat, nbad_off + sizeof(int), hipMemcpyDeviceToHost, stream));
  RW_HIP(hipMemcpyAsync(hs + bad_off, unanchored, sizeof(int), hipMemcpyDeviceToHost, stream));
  RW_HIP(hipStreamSynchronize(stream));
  double stat = 0.0;
  int bad = 0, nbad = 0;
  std::memcpy(&stat, hs, sizeof(double));
  std::memcpy(&bad, hs + bad_off, sizeof(int));
  std::memcpy(&nbad, hs + nbad_off, sizeof(int));
  RW_CHECK(!bad, RW_EUNANCHORED,
           "a connected component (edges with w >= 1e-30) holds no seed: the gamma = 0 system is singular");
  RW_CHECK(!nbad, RW_EINVAL, "basis column %d lies in the span of the null vector (column 0)", nbad);
  RW_CHECK(stat > 0.0, RW_ESINGULAR, "reduced seed system is singular to working precision (m = %d)", m);
  if (info) {
    info->m_used = m;
    info->eig_probes = probes;
    info->f_max = f_max;
    info->f_worst = f_worst;
    info->min_pivot = stat;
  }
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// Asynchronous variant (fixed m, seeds on the device): kernels only, no host read, no wait, no memset, so a
// caller can capture it into a HIP graph.  The caller's seeds are copied into the workspace with any entry
// out of range (node or label) replaced by 0, so no later kernel can index outside its arrays; such a
// seed, or seeds not strictly ascending, set a flag.  The last kernel writes the status word.
// ---------------------------------------------------------------------------------------------
__global__ void k_sanitize_seeds(const int64_t* node, const int32_t* label, int64_t S, int64_t N, int C,
                                 int64_t* node_out, int32_t* label_out, int* bad) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= S) return;
  const int64_t v = node[k];
  const int32_t l = label[k];
  const bool ok = v >= 0 && v < N && l >= 0 && l < C && (k == 0 || node[k - 1] < v);
  node_out[k] = (v >= 0 && v < N) ? v : 0;
  label_out[k] = (l >= 0 && l < C) ? l : 0;
  if (!ok) *bad = 1;
}

// status word: invalid seeds, then an unanchored component, then a basis column in the null vector's span,
// then a singular reduced system, else RW_OK
__global__ void k_solve_status(const int* flags, const double* stat, int32_t* status) {
  int st = RW_OK;
  if (flags[1]) st = RW_EINVAL;
  else if (flags[2]) st = RW_EUNANCHORED;
  else if (flags[0]) st = RW_EINVAL;
  else if (!(stat[0] > 0.0)) st = RW_ESINGULAR;
  *status = st;
}

// ---------------------------------------------------------------------------------------------
// Allocation-free variant (fixed m): the workspace lives in `scratch`, a file-scope device array that each
// GPU holds from module load to process end.  Host code never passes `scratch` itself (its name is a host
// stand-in there): the first call on a device, with that device current, takes its device address with
// hipGetSymbolAddress and keeps it per device.  The host side (seed sorting, status words) uses static
// arrays.  A process-wide lock serializes calls, and each call waits for its stream before it returns
// (also after a failure), so no two calls use the array at once.
// ---------------------------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int64_t kNoAllocMaxSeeds = 16384;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_na_mu;
static void* g_na_ptr[kNoAllocMaxDevices] = {};
static std::pair<int64_t, int32_t> g_na_pairs[kNoAllocMaxSeeds];
static int64_t g_na_nodes[kNoAllocMaxSeeds];
static int32_t g_na_labels[kNoAllocMaxSeeds];
static double g_na_stage[kStatusStageBytes / sizeof(double)];

static int noalloc_scratch(void** ptr) {
  int dev = -1;
  RW_HIP(hipGetDevice(&dev));
  RW_CHECK(dev >= 0 && dev < kNoAllocMaxDevices, RW_EINVAL, "device %d beyond the %d the library tracks", dev,
           kNoAllocMaxDevices);
  if (g_na_ptr[dev] == nullptr) {
    void* p = nullptr;
    RW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    RW_CHECK(p != nullptr, RW_EHIP, "no device address for the solve's scratch array");
    g_na_ptr[dev] = p;
  }
  *ptr = g_na_ptr[dev];
  return RW_OK;
}


// ---------------------------------------------------------------------------------------------
// gamma > 0 with prior probabilities (Sec. II-B, eqs. (15) and (17)).  With Lambda_g = Lambda + gamma I,
// G = B Q'_n (S x m), Z = Q'_n^T P_hat_n (m x C) and V = Lambda_g^{-1} Q'_s^T F_s, eq. (17) reduces, as the
// gamma = 0 system does, to the m x m system
//   (Lambda_g - Q'_s^T G) V = Q'_s^T [op_ss U_hat_s + gamma (U_hat_s + G Lambda_g^{-1} Z)]
// and eq. (15) to U_hat_n = Q'_n Y with Y = V + gamma Lambda_g^{-1} Z.  P_hat = D^{1/2} P (P under L).
// The choice of m from the priors (Sec. III-A2, eq. (25)) uses Z_hat = Q^T P_hat over all rows and the
// stored columns: g_k(m) = ||p_hat_k||^2 - sum_{j<m} Z_hat(j, k)^2 (Q orthonormal), for k = 0, r^d, 2 r^d, ...
// ---------------------------------------------------------------------------------------------
struct PriorWork {
  void* X;        // C x N (FP64 for an FP64 basis, else FP32): s_i P(k, i)
  double* Zh;     // ma x C: Q^T X over all rows and the stored columns
  double* Zp;     // m x C: Q'_n^T P_hat_n
  double* gdot;   // C: g^T X (exact null vector)
  double* xn2;    // C: ||X(k, :)||^2
  double* Xs;     // S x C: s_i P(k, i) at the seeds, FP64
  double* part;   // prep partials
  void* ppart;    // projection partials
  double* ptmp;   // kPairCols x C
};

static int prior_blocks(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (N + 2047) / 2048)); }

static size_t prior_layout(const Graph* g, int ma, int64_t S, int C, void* base, SolveWork* w, PriorWork* pw) {
  const size_t used = solve_layout(g, ma, S, C, base, w, false);
  Carver c(base ? static_cast<char*>(base) + ((used + 255) & ~size_t(255)) : nullptr);
  PriorWork t;
  t.X = c.take<double>((size_t)C * g->N);
  t.Zh = c.take<double>((size_t)ma * C);
  t.Zp = c.take<double>((size_t)ma * C);
  t.gdot = c.take<double>(C);
  t.xn2 = c.take<double>(C);
  t.Xs = c.take<double>((size_t)S * C);
  t.part = c.take<double>((size_t)prior_blocks(g->N) * C * 2);
  t.ppart = c.take<char>(project_block_partial_bytes(g->N, ma, C));
  t.ptmp = c.take<double>((size_t)kPairCols * C);
  if (pw) *pw = t;
  return ((used + 255) & ~size_t(255)) + c.used;
}

// X(k, i) = s_i P(k, i); block b sums g_i X(k, i) and X(k, i)^2 over its node range (fixed order)
template <typename TP, typename TX>
__global__ __launch_bounds__(256) void k_prior_prep(const TP* P, int64_t N, int C, const double* degree,
                                                    const double* sums, int normalized, TX* X, double* part) {
  __shared__ double sh[4][2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t per = (N + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = blockIdx.x * per, i1 = min(N, i0 + per);
  for (int k = 0; k < C; ++k) {
    double a = 0.0, b = 0.0;
    for (int64_t i = i0 + tid; i < i1; i += 256) {
      const double sc = normalized ? sqrt(degree[i]) : 1.0;
      const double x = sc * (double)P[(int64_t)k * N + i];
      const TX xs = (TX)x;
      X[(int64_t)k * N + i] = xs;
      a += ghat64(degree, sums, normalized, N, i) * (double)xs;
      b += (double)xs * (double)xs;
    }
    a = wave_sum64(a);
    b = wave_sum64(b);
    __syncthreads();
    if (lane == 0) {
      sh[wave][0] = a;
      sh[wave][1] = b;
    }
    __syncthreads();
    if (tid < 2)
      part[((int64_t)blockIdx.x * C + k) * 2 + tid] = (sh[0][tid] + sh[1][tid]) + (sh[2][tid] + sh[3][tid]);
  }
}

__global__ void k_prior_norms(const double* part, int nb, int C, double* gdot, double* xn2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= C) return;
  double a = 0.0, b = 0.0;
  for (int q = 0; q < nb; ++q) {
    a += part[((int64_t)q * C + k) * 2];
    b += part[((int64_t)q * C + k) * 2 + 1];
  }
  gdot[k] = a;
  xn2[k] = b;
}

// Xs(s, k) = s_i P(k, i) at seed s (node i), FP64
template <typename TP>
__global__ void k_prior_xs(const TP* P, int64_t N, int C, const int64_t* seeds, int64_t S, const double* degree,
                           int normalized, double* Xs) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= S * C) return;
  const int64_t s = t % S, k = t / S;
  const int64_t i = seeds[s];
  Xs[t] = (normalized ? sqrt(degree[i]) : 1.0) * (double)P[k * N + i];
}

// Zp(j, k) = q'_j^T X(k, :) over the non-seed rows: the full-row projection in the FP64 basis (q'_0 = g,
// q'_j = (q_j - g c_j) / n_j) less the seed rows' part
__global__ void k_prior_z(int m, int ma, int C, int64_t S, const double* Zh, const double* gdot, const double* cn,
                          const double* Qs, const double* Xs, double* Zp) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * C) return;
  const int j = (int)(t % m), k = (int)(t / m);
  double z = j == 0 ? gdot[k] : (Zh[j + (int64_t)k * ma] - cn[j] * gdot[k]) / cn[m + j];
  for (int64_t s = 0; s < S; ++s) z -= Qs[s + (int64_t)j * S] * Xs[s + (int64_t)k * S];
  Zp[t] = z;
}

// Hs(s, k) += gamma (U_hat_s(s, k) + sum_j G(s, j) Zp(j, k) / (lambda_j + gamma))
__global__ void k_prior_rhs(int m, int C, int64_t S, const double* GB, const double* Us, const double* lambda,
                            double gamma, const double* Zp, double* Hs) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= S * C) return;
  const int64_t s = t % S, k = t / S;
  double acc = 0.0;
  for (int j = 0; j < m; ++j) acc += GB[s + (int64_t)j * S] * Zp[j + k * m] / (lambda[j] + gamma);
  Hs[t] += gamma * (Us[t] + acc);
}

// Y(j, k) += gamma Zp(j, k) / (lambda_j + gamma)
__global__ void k_prior_finish(int m, int C, const double* lambda, double gamma, const double* Zp, double* Y) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * C) return;
  const int j = (int)(t % m);
  Y[t] += gamma * Zp[t] / (lambda[j] + gamma);
}

static int prior_solve_impl(rw_graph h, const void* Q, int q_dtype, const double* lambda, int ma,
                            const int64_t* nodes, const int32_t* labels, int64_t S, int C, double gamma,
                            const void* prior, int prior_dtype, double eps, int r, void* U, const SolveWork& w,
                            const PriorWork& pw, hipStream_t stream, rw_solve_info* info) {
  const Graph* g = &h->g;
  RW_HIP(hipMemcpyAsync(w.seeds, nodes, S * sizeof(int64_t), hipMemcpyHostToDevice, stream));
  RW_HIP(hipMemcpyAsync(w.labels, labels, S * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  k_clear_map<<<nblocks(g->N, 256), 256, 0, stream>>>(w.map, g->N);
  RW_LAUNCH_CHECK();
  k_set_map<<<nblocks(S, 256), 256, 0, stream>>>(w.map, w.seeds, w.labels, S);
  RW_LAUNCH_CHECK();
  RW_TRY(seed_gather(g, Q, q_dtype, ma, w, S, C, stream));
  RW_TRY(fill_i32(w.nbad, 1, 0, stream));
  // X = s P, its projection on the stored columns, g^T X and ||X||^2
  const bool x64 = q_dtype == RW_F64;
  const int nb = prior_blocks(g->N);
#define RW_PREP(TP, TX)                                                                                      \
  k_prior_prep<TP, TX><<<nb, 256, 0, stream>>>(static_cast<const TP*>(prior), g->N, C, g->degree, g->sums,    \
                                               g->normalized, static_cast<TX*>(pw.X), pw.part)
  if (prior_dtype == RW_F64) {
    if (x64) RW_PREP(double, double);
    else RW_PREP(double, float);
  } else {
    if (x64) RW_PREP(float, double);
    else RW_PREP(float, float);
  }
#undef RW_PREP
  RW_LAUNCH_CHECK();
  k_prior_norms<<<nblocks(C, 256), 256, 0, stream>>>(pw.part, nb, C, pw.gdot, pw.xn2);
  RW_LAUNCH_CHECK();
  RW_TRY(project_block(Q, q_dtype, g->N, ma, pw.X, C, pw.Zh, pw.ppart, pw.ptmp, stream));
  // choice of m (eq. (25)) on the sampled labels
  int m = ma;
  double gmax = 0.0, gworst = 0.0;
  if (eps > 0.0) {
    int step = 1;
    for (int q = 0; q < g->ndim; ++q) step *= r;
    const int ns = (C + step - 1) / step;
    void* stage = nullptr;
    RW_TRY(host_stage(((size_t)ma * C + C + 1) * sizeof(double), &stage));
    double* hz = static_cast<double*>(stage);
    RW_HIP(hipMemcpyAsync(hz, pw.Zh, (size_t)ma * C * sizeof(double), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipMemcpyAsync(hz + (size_t)ma * C, pw.xn2, C * sizeof(double), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipMemcpyAsync(hz + (size_t)ma * C + C, g->sums, sizeof(double), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipStreamSynchronize(stream));
    gmax = eps * eps * (g->normalized ? hz[(size_t)ma * C + C] : (double)g->N);
    std::vector<double> gk((size_t)ns);
    for (int q = 0; q < ns; ++q) gk[q] = hz[(size_t)ma * C + (size_t)q * step];
    m = ma;
    for (int mm = 1; mm <= ma; ++mm) {
      double worst = 0.0;
      for (int q = 0; q < ns; ++q) {
        const double z = hz[(mm - 1) + (size_t)q * step * ma];
        gk[q] -= z * z;
        worst = std::max(worst, gk[q]);
      }
      gworst = worst;
      if (mm >= 2 && worst <= gmax) {
        m = mm;
        break;
      }
    }
  }
  // the FP64 basis of the first m columns, the projection of P_hat_n on it, and the reduced system
  RW_TRY(null_stats(g, Q, q_dtype, m, w.npart, w.cn, w.nbad, stream));
  k_seed_correct<<<nblocks(S * m, 256), 256, 0, stream>>>(w.Qs, w.GB, w.gs, w.Bg, w.cn, S, m);
  RW_LAUNCH_CHECK();
  if (prior_dtype == RW_F64)
    k_prior_xs<double><<<nblocks(S * C, 256), 256, 0, stream>>>(static_cast<const double*>(prior), g->N, C, w.seeds,
                                                                S, g->degree, g->normalized, pw.Xs);
  else
    k_prior_xs<float><<<nblocks(S * C, 256), 256, 0, stream>>>(static_cast<const float*>(prior), g->N, C, w.seeds,
                                                               S, g->degree, g->normalized, pw.Xs);
  RW_LAUNCH_CHECK();
  k_prior_z<<<nblocks((int64_t)m * C, 256), 256, 0, stream>>>(m, ma, C, S, pw.Zh, pw.gdot, w.cn, w.Qs, pw.Xs, pw.Zp);
  RW_LAUNCH_CHECK();
  k_prior_rhs<<<nblocks(S * C, 256), 256, 0, stream>>>(m, C, S, w.GB, w.Us, lambda, gamma, pw.Zp, w.Hs);
  RW_LAUNCH_CHECK();
  k_reduced<<<reduced_grid(m, C), 256, 0, stream>>>(m, C, S, w.Qs, w.GB, w.Hs, lambda, gamma, w.K,
                                                                     w.Y);
  RW_LAUNCH_CHECK();
  RW_TRY(lu_solve(w.K, m, w.Y, C, w.stat, stream));
  k_prior_finish<<<nblocks((int64_t)m * C, 256), 256, 0, stream>>>(m, C, lambda, gamma, pw.Zp, w.Y);
  RW_LAUNCH_CHECK();
  RW_TRY(solve_coeffs(w.Y, m, C, w.cn, g, stream));
  RW_TRY(reconstruct(g, Q, q_dtype, m, w.Y, C, w.map, U, stream));
  // stat and the null-column flag are adjacent in the workspace: one copy
  const size_t nbad_off = reinterpret_cast<const char*>(w.nbad) - reinterpret_cast<const char*>(w.stat);
  void* stage = nullptr;
  RW_TRY(host_stage(nbad_off + sizeof(int), &stage));
  const char* hs = static_cast<const char*>(stage);
  RW_HIP(hipMemcpyAsync(stage, w.stat, nbad_off + sizeof(int), hipMemcpyDeviceToHost, stream));
  RW_HIP(hipStreamSynchronize(stream));
  double stat = 0.0;
  int nbad = 0;
  std::memcpy(&stat, hs, sizeof(double));
  std::memcpy(&nbad, hs + nbad_off, sizeof(int));
  RW_CHECK(!nbad, RW_EINVAL, "basis column %d lies in the span of the null vector (column 0)", nbad);
  RW_CHECK(stat > 0.0, RW_ESINGULAR, "reduced seed system is singular to working precision (m = %d)", m);
  if (info) {
    info->m_used = m;
    info->eig_probes = 0;
    info->f_max = gmax;
    info->f_worst = gworst;
    info->min_pivot = stat;
  }
  return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_solve_seeds_noalloc(rw_graph h, const void* Q, int q_dtype, const double* lambda, int m,
                           const int64_t* seed_node, const int32_t* seed_label, int64_t S_in, int C, void* U,
                           hipStream_t stream, rw_solve_info* info) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  const Graph* g = &h->g;
  RW_CHECK(Q != nullptr && lambda != nullptr && U != nullptr, RW_EINVAL, "null pointer argument");
  RW_CHECK(q_dtype_ok(q_dtype), RW_EINVAL, "bad Q dtype");
  RW_CHECK(m >= 2 && m <= g->N, RW_EINVAL, "m = %d out of range", m);
  RW_CHECK(S_in >= 1, RW_EINVAL, "at least one seed is required");
  RW_CHECK(S_in <= kNoAllocMaxSeeds, RW_EWORKSPACE, "%lld seeds exceed the %lld of the allocation-free solve",
           (long long)S_in, (long long)kNoAllocMaxSeeds);
  const size_t need = solve_layout(g, m, S_in, C, nullptr, nullptr, false);
  RW_CHECK(need <= kNoAllocScratchBytes, RW_EWORKSPACE,
           "the solve needs %zu bytes of workspace, above the %zu of the allocation-free entry point", need,
           kNoAllocScratchBytes);
  std::lock_guard<std::mutex> lock(g_na_mu);
  void* base = nullptr;
  RW_TRY(noalloc_scratch(&base));
  int64_t S = 0;
  RW_TRY(host_seeds_into(g, seed_node, seed_label, S_in, C, g_na_pairs, g_na_nodes, g_na_labels, &S));
  RW_CHECK(S < g->N, RW_EINVAL, "every node is a seed");
  SolveWork w;
  solve_layout(g, m, S_in, C, base, &w, false);
  const int st = solve_impl(h, Q, q_dtype, lambda, m, g_na_nodes, g_na_labels, S, S_in, C, 0.0, U, w, stream, info,
                            g_na_stage);
  if (st != RW_OK) (void)hipStreamSynchronize(stream);   // nothing of a failed call still uses the array
  return st;
}

int rw_solve_seeds_async(rw_graph h, const void* Q, int q_dtype, const double* lambda, int m,
                         const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C, void* U, void* work,
                         size_t work_bytes, int32_t* status, hipStream_t stream) {
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  const Graph* g = &h->g;
  RW_CHECK(Q != nullptr && lambda != nullptr && U != nullptr && work != nullptr && status != nullptr &&
               seed_node != nullptr && seed_label != nullptr,
           RW_EINVAL, "null pointer argument");
  RW_CHECK(q_dtype_ok(q_dtype), RW_EINVAL, "bad Q dtype");
  RW_CHECK(m >= 2 && m <= g->N, RW_EINVAL, "m = %d out of range", m);
  RW_CHECK(S >= 1 && S < g->N, RW_EINVAL, "S = %lld out of range", (long long)S);
  RW_CHECK(C >= 1 && C <= 255, RW_EINVAL, "C must be in [1, 255] (got %d)", C);
  RW_CHECK(g->cc_valid, RW_EINVAL,
           "the graph's components are not current: call rw_graph_components after the last build or edit");
  SolveWork w;
  const size_t need = solve_layout(g, m, S, C, work, &w, false);
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "solve workspace too small: %zu < %zu", work_bytes, need);
  int* flags = w.nbad;   // [0] basis column in the null span, [1] invalid seeds, [2] unanchored
  RW_TRY(fill_i32(flags, 3, 0, stream));
  k_sanitize_seeds<<<nblocks(S, 256), 256, 0, stream>>>(seed_node, seed_label, S, g->N, C, w.seeds, w.labels,
                                                        flags + 1);
  RW_LAUNCH_CHECK();
  RW_TRY(anchor_launch_async(g, w.seeds, S, w.anc, flags + 2, stream));
  k_clear_map<<<nblocks(g->N, 256), 256, 0, stream>>>(w.map, g->N);
  RW_LAUNCH_CHECK();
  k_set_map<<<nblocks(S, 256), 256, 0, stream>>>(w.map, w.seeds, w.labels, S);
  RW_LAUNCH_CHECK();
  RW_TRY(seed_gather(g, Q, q_dtype, m, w, S, C, stream));
  RW_TRY(null_stats(g, Q, q_dtype, m, w.npart, w.cn, flags, stream));
  k_seed_correct<<<nblocks(S * m, 256), 256, 0, stream>>>(w.Qs, w.GB, w.gs, w.Bg, w.cn, S, m);
  RW_LAUNCH_CHECK();
  k_reduced<<<reduced_grid(m, C), 256, 0, stream>>>(m, C, S, w.Qs, w.GB, w.Hs, lambda, 0.0, w.K,
                                                                     w.Y);
  RW_LAUNCH_CHECK();
  RW_TRY(lu_solve(w.K, m, w.Y, C, w.stat, stream));
  RW_TRY(solve_coeffs(w.Y, m, C, w.cn, g, stream));
  RW_TRY(reconstruct(g, Q, q_dtype, m, w.Y, C, w.map, U, stream));
  k_solve_status<<<1, 1, 0, stream>>>(flags, w.stat, status);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

int rw_solve_workspace_bytes(rw_graph h, int m_avail, int64_t S, int C, size_t* bytes) {
  RW_CHECK(h != nullptr && bytes != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(m_avail >= 2 && S >= 1 && C >= 1, RW_EINVAL, "bad sizes");
  *bytes = solve_layout(&h->g, m_avail, S, C, nullptr, nullptr);
  return RW_OK;
}

int rw_solve_seeds(rw_graph h, const void* Q, int q_dtype, const double* lambda, int m_avail,
                   const int64_t* seed_node, const int32_t* seed_label, int64_t S_in, int C, double eps, void* U,
                   void* work, size_t work_bytes, hipStream_t stream, rw_solve_info* info) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  const Graph* g = &h->g;
  RW_CHECK(Q != nullptr && lambda != nullptr && U != nullptr && work != nullptr, RW_EINVAL, "null pointer argument");
  RW_CHECK(q_dtype_ok(q_dtype), RW_EINVAL, "bad Q dtype");
  RW_CHECK(m_avail >= 2 && m_avail <= g->N, RW_EINVAL, "m_avail = %d out of range", m_avail);
  RW_CHECK(S_in >= 1, RW_EINVAL, "at least one seed is required");
  std::vector<std::pair<int64_t, int32_t>> v((size_t)S_in);
  std::vector<int64_t> nodes((size_t)S_in);
  std::vector<int32_t> labels((size_t)S_in);
  int64_t S = 0;
  RW_TRY(host_seeds_into(g, seed_node, seed_label, S_in, C, v.data(), nodes.data(), labels.data(), &S));
  RW_CHECK(S < g->N, RW_EINVAL, "every node is a seed");
  SolveWork w;
  size_t need = solve_layout(g, m_avail, S_in, C, work, &w);  // sized for S_in >= S
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "solve workspace too small: %zu < %zu", work_bytes, need);
  return solve_impl(h, Q, q_dtype, lambda, m_avail, nodes.data(), labels.data(), S, S_in, C, eps, U, w, stream, info,
                    nullptr);
}

int rw_solve_prior_workspace_bytes(rw_graph h, int m_avail, int64_t S, int C, size_t* bytes) {
  RW_CHECK(h != nullptr && bytes != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(m_avail >= 2 && S >= 1 && C >= 1, RW_EINVAL, "bad sizes");
  *bytes = prior_layout(&h->g, m_avail, S, C, nullptr, nullptr, nullptr);
  return RW_OK;
}

int rw_solve_seeds_prior(rw_graph h, const void* Q, int q_dtype, const double* lambda, int m_avail,
                         const int64_t* seed_node, const int32_t* seed_label, int64_t S_in, int C, double gamma,
                         const void* prior, int prior_dtype, double eps, int r, void* U, void* work,
                         size_t work_bytes, hipStream_t stream, rw_solve_info* info) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  const Graph* g = &h->g;
  RW_CHECK(Q != nullptr && lambda != nullptr && U != nullptr && work != nullptr && prior != nullptr, RW_EINVAL,
           "null pointer argument");
  RW_CHECK(q_dtype_ok(q_dtype), RW_EINVAL, "bad Q dtype");
  RW_CHECK(prior_dtype == RW_F64 || prior_dtype == RW_F32, RW_EINVAL, "priors are F64 or F32");
  RW_CHECK(gamma > 0.0 && std::isfinite(gamma), RW_EINVAL, "gamma must be positive (got %g)", gamma);
  RW_CHECK(m_avail >= 2 && m_avail <= g->N, RW_EINVAL, "m_avail = %d out of range", m_avail);
  RW_CHECK(eps <= 0.0 || (r >= 1 && r <= 64), RW_EINVAL, "label sampling step r = %d out of range", r);
  RW_CHECK(S_in >= 1, RW_EINVAL, "at least one seed is required");
  std::vector<std::pair<int64_t, int32_t>> v((size_t)S_in);
  std::vector<int64_t> nodes((size_t)S_in);
  std::vector<int32_t> labels((size_t)S_in);
  int64_t S = 0;
  RW_TRY(host_seeds_into(g, seed_node, seed_label, S_in, C, v.data(), nodes.data(), labels.data(), &S));
  RW_CHECK(S < g->N, RW_EINVAL, "every node is a seed");
  SolveWork w;
  PriorWork pw;
  const size_t need = prior_layout(g, m_avail, S_in, C, work, &w, &pw);
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "prior solve workspace too small: %zu < %zu", work_bytes, need);
  return prior_solve_impl(h, Q, q_dtype, lambda, m_avail, nodes.data(), labels.data(), S, C, gamma, prior,
                          prior_dtype, eps, r, U, w, pw, stream, info);
}

}  // extern "C"
