// Symmetric eigendecomposition through a tridiagonal form, for one matrix of order n <= 256 (batches of
// matrices up to order 199):
//   1. Householder reduction A = U T U^T (Golub & Van Loan Sec. 8.3.1) in one workgroup: up to order 224
//      with the matrix in registers (k_tridiag_reg, below); above, with the packed lower triangle in LDS:
//      per column, one wave forms the reflector (the next column's while the other waves finish the
//      rank-2 update), 4 to 16 lanes per row form p = tau A22 v, every wave forms K = tau/2 p^T v, and all
//      threads apply the rank-2 update A22 -= v w^T + w v^T with w = p - K v; the first n - 199 columns
//      are reduced on a full copy in global memory (L2-resident) and the rest in LDS;
//   2. eigenvalues of T by multisection on Sturm counts (Sec. 8.4.1), kBisThreads points per pass, one
//      workgroup per eigenvalue (the interval shrinks kBisThreads + 1-fold per pass);
//   3. eigenvectors of T by inverse iteration with the LDL^T factorization of T - lambda I (one lane
//      per eigenvector, three solves, in LDS);
//   4. V = U Z, the reflectors applied to each eigenvector column (one wave per column).
// Inverse iteration gives orthogonal vectors only when eigenvalues are separated: the vectors of a
// cluster (successive eigenvalues closer than 1e-6 |T|) are computed again, in order, by inverse
// iteration with Gram-Schmidt against the cluster's earlier vectors in every step (the approach of
// LAPACK's dstein).  The driver reports RW_ENOCONV only for a cluster of more than kTriClusterMax vectors
// or one whose vectors vanish under the orthogonalization; the caller then uses the Jacobi solver.
// All arithmetic is FP64.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "rw_internal.h"

namespace rw {

__device__ __forceinline__ int tr_lo(int i, int j, int n) { return j * n - ((j * (j - 1)) >> 1) + (i - j); }  // i >= j

static size_t tridiag_lds_bytes(int n) { return ((size_t)n * (n + 1) / 2 + 2 * (size_t)n) * sizeof(double); }
constexpr int kTriLdsMax = 199;   // the largest order whose packed triangle (and two vectors) fit in LDS

static size_t invit_lds_bytes(int n, int tpb);
bool tridiag_batch_fits(int n) {   // n <= 199: the batched range (inverse iteration stages 32 vectors in LDS)
  return n >= 3 && n <= kTriLdsMax && tridiag_lds_bytes(n) <= kLdsLimit && invit_lds_bytes(n, 32) <= kLdsLimit;
}
bool tridiag_fits(int n) { return n >= 3 && n <= 256; }
static_assert((size_t)kTriLdsMax * (kTriLdsMax + 1) / 2 * 8 + 2 * kTriLdsMax * 8 <= kLdsLimit, "LDS");

// work (doubles): reflectors n x n (reflector k in column k, entries 0..n-k-2, first entry 1), tau n, d n,
// e n, lambda n, Z n x n (Z(j, i) = entry j of eigenvector i at j * n + i), LDL^T scratch 2 n x n, flag
size_t tridiag_work_count(int n) { return (size_t)n * n * 4 + (size_t)n * 6 + 8; }

struct TriBufs {
  double *refl, *tau, *d, *e, *lam, *Z, *Lf, *Df, *flag;
};

static TriBufs tri_bufs(double* work, int n) {
  TriBufs b;
  const size_t nn = (size_t)n * n;
  b.refl = work;
  b.tau = b.refl + nn;
  b.d = b.tau + n;
  b.e = b.d + n;
  b.lam = b.e + n;
  b.Z = b.lam + n;
  b.Lf = b.Z + nn;
  b.Df = b.Lf + nn;
  b.flag = b.Df + nn;
  return b;
}

// sum over the 64 lanes of a wave, the same in every lane (DPP within rows, rows in a fixed order)
__device__ __forceinline__ double tr_wave_sum(double v) { return wave_sum64(v); }

// 1. Householder tridiagonalization (lower): reflector k maps A(k+1:n, k) to beta e1
// Workgroup b reduces matrix b of a batch: order sz.n[b], leading dimension lda, matrices strideA apart;
// its reflectors, tau, d and e sit nmax^2 or nmax entries apart per matrix.
// Orders above kTriLdsMax (one matrix only): the first t0 = n - nl columns are reduced on a full symmetric
// copy in global memory (Aw, n x n column-major, L2-resident: per step a thread-per-row matrix-vector
// product and rank-2 update, coalesced along the columns), then the trailing triangle of order nl moves
// to LDS and the reduction continues there with local indices.
__global__ __launch_bounds__(1024) void k_tridiag(const double* A, int lda, int64_t strideA, TriSizes sz, int nmax,
                                                  double* refl, double* tau, double* d, double* e, double* flag,
                                                  double* Aw, int t0) {
  const int b = blockIdx.x, n = sz.n[b];
  if (b == 0 && threadIdx.x == 0) flag[0] = 0.0;   // the flag of the cluster pass that follows
  A += b * strideA;
  refl += (int64_t)b * nmax * nmax;
  tau += (int64_t)b * nmax;
  d += (int64_t)b * nmax;
  e += (int64_t)b * nmax;
  extern __shared__ double sA[];   // packed lower triangle of the trailing order nl, column-major
  const int nl = n - t0;
  double* v = sA + nl * (nl + 1) / 2;
  double* p = v + nl;
  __shared__ double s_tau[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // reflector k from the column below the diagonal x[0 .. m) (m = n - k - 1), by wave 0: v_k into vk, its
  // entries to refl, tau, e, and tau for the workgroup in s_tau[k & 1]; the diagonal entry dk to d
  auto reflector = [&](int k, const double* x, int xstride, double dk, double* vk) {
    const int m = n - k - 1;
    double xs[4];
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      xs[q] = i < m ? x[(int64_t)i * xstride] : 0.0;
      if (i >= 1) ss += xs[q] * xs[q];
    }
    ss = tr_wave_sum(ss);
    const double x0 = __shfl(xs[0], 0);
    double beta, tk, scale;
    if (ss == 0.0) {   // already reduced: no reflection
      tk = 0.0;
      beta = x0;
      scale = 0.0;
    } else {
      const double nrm = sqrt(x0 * x0 + ss);
      beta = x0 >= 0.0 ? -nrm : nrm;
      tk = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (i < m) {
        const double vi = i == 0 ? 1.0 : xs[q] * scale;
        vk[i] = vi;
        refl[(int64_t)k * n + i] = vi;
      }
    }
    if (lane == 0) {
      s_tau[k & 1] = tk;
      tau[k] = tk;
      e[k] = beta;
      d[k] = dk;
    }
  };
  if (t0 > 0) {
    // ---- global phase: columns 0 .. t0-1 on the full copy Aw (ld n); vectors in the LDS region ----
    double* gv = sA;            // two reflector vectors (256 each)
    double* gp = sA + 512;      // p (256)
    double* gred = sA + 768;    // matrix-vector partials, 4 x 256
    for (int t = tid; t < n * n; t += blockDim.x) {
      const int i = t % n, j = t / n;
      Aw[t] = 0.5 * (A[i + (int64_t)j * lda] + A[j + (int64_t)i * lda]);
    }
    __syncthreads();
    for (int k = 0; k < t0; ++k) {
      const int m = n - k - 1;
      double* vk = gv + 256 * (k & 1);
      const double* col = Aw + (int64_t)k * n + (k + 1);   // A(k+1 .., k)
      if (wave == 0) reflector(k, col, 1, Aw[(int64_t)k * n + k], vk);
      __syncthreads();
      const double tk = s_tau[k & 1];
      if (tk == 0.0) continue;   // uniform
      // p = tk A22 v: thread (r, g) sums the columns c = g, g + 4, .. of row r, then the four groups in order
      const int r = tid & 255, g = tid >> 8;
      double* A22 = Aw + (int64_t)(k + 1) * n + (k + 1);   // A22(r, c) at r + c n
      if (r < m) {
        double acc = 0.0;
        for (int c = g; c < m; c += 4) acc += A22[r + (int64_t)c * n] * vk[c];
        gred[g * 256 + r] = acc;
      }
      __syncthreads();
      if (tid < m) gp[tid] = tk * ((gred[tid] + gred[256 + tid]) + (gred[512 + tid] + gred[768 + tid]));
      __syncthreads();
      // K = tk / 2 p^T v, then A22 -= v w^T + w v^T with w = p - K v (the full square: both triangles)
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        if (i < m) s += gp[i] * vk[i];
      }
      const double K = 0.5 * tk * tr_wave_sum(s);
      if (r < m) {
        const double vr = vk[r], wr = gp[r] - K * vr;
        for (int c = g; c < m; c += 4) {
          const double vc = vk[c], wc = gp[c] - K * vc;
          A22[r + (int64_t)c * n] -= vr * wc + wr * vc;
        }
      }
      __syncthreads();
    }
    // the trailing lower triangle (order nl) into LDS
    for (int t = tid; t < nl * nl; t += blockDim.x) {
      const int i = t % nl, j = t / nl;
      if (i >= j) sA[tr_lo(i, j, nl)] = Aw[(t0 + i) + (int64_t)(t0 + j) * n];
    }
    __syncthreads();
  } else {
    for (int t = tid; t < n * n; t += blockDim.x) {
      const int i = t % n, j = t / n;
      if (i >= j) sA[tr_lo(i, j, n)] = 0.5 * (A[i + (int64_t)j * lda] + A[j + (int64_t)i * lda]);
    }
    __syncthreads();
  }
  // ---- LDS phase: local step kl = k - t0 on the packed triangle of order nl ----
  // v_kl lives in the packed slots of local column kl-1 below its diagonal (nl - kl entries, dead once that
  // reflector is formed), v_0 in its own array: so reflector kl+1 can be formed while step kl still reads v_kl
  auto vbuf = [&](int kl) -> double* { return kl == 0 ? v : sA + tr_lo(kl, kl - 1, nl); };
  auto reflector_lds = [&](int kl, double* vk) {
    reflector(kl + t0, sA + tr_lo(kl + 1, kl, nl), 1, sA[tr_lo(kl, kl, nl)], vk);
  };
  bool ahead = false;   // reflector kl already formed during step kl-1 (uniform)
  for (int kl = 0; kl < nl - 2; ++kl) {
    const int k = kl + t0;
    const int m = n - k - 1;   // length of the column below the diagonal
    double* vk = vbuf(kl);
    if (!ahead) {
      if (wave == 0) reflector_lds(kl, vk);
      lds_barrier();
    }
    const double tk = s_tau[k & 1];
    ahead = false;
    if (tk == 0.0) continue;   // uniform
    // p = tk A22 v (A22 = A(kl+1:nl, kl+1:nl), symmetric, lower stored): L lanes per row (one DPP quad, half
    // row or row), more lanes as the block shrinks so that more waves share the rows
    {
      const int LS = m > 128 ? 2 : (m > 64 ? 3 : 4), L = 1 << LS;
      const int tri = (L * (L + 1)) >> 1;
      for (int rb = 0; rb < m; rb += (int)(blockDim.x >> LS)) {   // uniform
        const int r = rb + (tid >> LS), sub = tid & (L - 1);
        double acc = 0.0;
        if (r < m) {
          const int R = kl + 1 + r;
          int j = sub;
          // j <= r: row R of the lower triangle, A(R, C) with C = kl + 1 + j; the packed address advances by
          // colstart(C + L) - colstart(C) - L = L (nl - C) - L (L + 1) / 2
          int C = kl + 1 + j, addr = tr_lo(R, C, nl);
          for (; j <= r; j += L, C += L) {
            acc += sA[addr] * vk[j];
            addr += L * (nl - C) - tri;
          }
          // j > r: column R, A(C, R), consecutive in C
          addr = tr_lo(kl + 1 + j, R, nl);
          for (; j < m; j += L, addr += L) acc += sA[addr] * vk[j];
        }
        if (LS == 2) {
          acc = quad_sum(acc);
        } else if (LS == 3) {
          acc = quad_sum(acc);
          acc += dpp_mov<0x141>(acc);   // row_half_mirror: the eight lanes of a half row
        } else {
          acc = row16_sum(acc);
        }
        if (sub == 0 && r < m) p[r] = tk * acc;
      }
    }
    lds_barrier();
    // K = tk / 2 p^T v (every wave), then A22 -= v w^T + w v^T with w = p - K v
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (i < m) s += p[i] * vk[i];
    }
    const double K = 0.5 * tk * tr_wave_sum(s);
    const int tx = tid & 31, ty = tid >> 5;
    auto update_col = [&](int jj) {
      const double vj = vk[jj], wj = p[jj] - K * vj;
      int addr = tr_lo(kl + 1 + jj + tx, kl + 1 + jj, nl);
      for (int ii = jj + tx; ii < m; ii += 32, addr += 32) {
        const double vi = vk[ii], wi = p[ii] - K * vi;
        sA[addr] -= vi * wj + wi * vj;
      }
    };
    if (ty < m) update_col(ty);
    // look-ahead: column 0 of A22 (local column kl+1) was updated by lanes 0-31 of wave 0 just now, so wave 0
    // forms reflector kl+1 while the other waves finish the update
    const bool la = kl + 1 < nl - 2;
    if (la && wave == 0) reflector_lds(kl + 1, vbuf(kl + 1));
    // the later columns in reverse order of ty, so that wave 0, which also formed the reflector, gets the
    // shortest of each group of 32
    for (int jj = (31 - ty) + 32; jj < m; jj += 32) update_col(jj);
    ahead = la;
    lds_barrier();
  }
  __syncthreads();
  if (tid == 0) {
    d[n - 2] = sA[tr_lo(nl - 2, nl - 2, nl)];
    d[n - 1] = sA[tr_lo(nl - 1, nl - 1, nl)];
    e[n - 2] = sA[tr_lo(nl - 1, nl - 2, nl)];
    e[n - 1] = 0.0;
    tau[n - 2] = 0.0;
    tau[n - 1] = 0.0;
  }
}

// 1'. The same reduction with the matrix in registers, for orders up to kTriRegMax: 512 threads, thread
// (lane, wave) holds A(i, j) for the rows i = lane + 64 s (s < RS) and the columns j = wave + 8 t (t < CS),
// both triangles, so that no step reads or writes the matrix in LDS.  Per column k:
//   * the wave that holds column k (wave k mod 8) forms reflector k from its registers at the end of step
//     k-1, once its update is done; v (zero at i <= k and i >= n, 1 at k+1) goes to LDS (two buffers, by the
//     parity of k);
//   * barrier; each thread sums A(i, j) v_j over its columns for each of its rows (v_j by a row broadcast
//     from a copy of v that holds the wave's columns in the 16 lanes of each row); the row partials of the
//     eight waves go to LDS;
//   * barrier; 256 threads add a row's eight partials in a fixed order: p = tau A22 v (zero at i <= k);
//   * barrier; every wave forms K = tau/2 p^T v and w = p - K v, and each thread applies
//     A -= v w^T + w v^T to its elements.  Elements in finished rows or columns see v = w = 0 there and keep
//     their values; column slots left of the step's group of eight columns and row slots above it are
//     skipped.
// Outputs as k_tridiag: reflector k in refl[k n ..], tau, d and e.
constexpr int kTriRegMax = 224;
constexpr int kTriRegThreads = 512;
static size_t tridiag_reg_lds_bytes() { return (size_t)(2 * 256 + 256 + 8 * 256) * sizeof(double); }

template <int RS, int CS>
__global__ __launch_bounds__(kTriRegThreads) void k_tridiag_reg(const double* A, int lda, int64_t strideA,
                                                                TriSizes sz, int nmax, double* refl, double* tau,
                                                                double* d, double* e, double* flag) {
  static_assert(RS >= 1 && RS <= 4 && 8 * CS <= 64 * RS, "layout");
  const int b = blockIdx.x, n = sz.n[b];
  if (b == 0 && threadIdx.x == 0) flag[0] = 0.0;   // the flag of the cluster pass that follows
  A += b * strideA;
  refl += (int64_t)b * nmax * nmax;
  tau += (int64_t)b * nmax;
  d += (int64_t)b * nmax;
  e += (int64_t)b * nmax;
  extern __shared__ double sT[];
  __shared__ double s_tau[2];
  // the wave index as a uniform value, so that the slot tests below are scalar branches
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double a[RS][CS];
  // 0.5 (A + A^T), straight from memory (A(i, j) with consecutive rows across lanes; A(j, i) one row per lane,
  // from L2: the matrix was just written)
#pragma unroll
  for (int s = 0; s < RS; ++s)
#pragma unroll
    for (int t = 0; t < CS; ++t) {
      const int i = lane + 64 * s, j = wave + 8 * t;
      a[s][t] = (i < n && j < n) ? 0.5 * (A[i + (int64_t)j * lda] + A[j + (int64_t)i * lda]) : 0.0;
    }
  double* sv = sT;             // v of the step, two buffers of 256
  double* sp = sT + 512;       // p (256)
  double* sPr = sT + 768;      // row partials, 8 x 256
  // reflector k from x = column k (rows lane + 64 s), by the wave holding it: v to sv[k & 1], tau to s_tau[k & 1]
  auto reflector = [&](int k, const double (&x)[RS]) {
    double ss = 0.0, xk = x[0], xk1 = x[0];
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int i = lane + 64 * s;
      if (i >= k + 2 && i < n) ss += x[s] * x[s];
      if (s == (k >> 6)) xk = x[s];
      if (s == ((k + 1) >> 6)) xk1 = x[s];
    }
    ss = wave_sum64(ss);
    const double dk = lane_read(xk, k & 63), x0 = lane_read(xk1, (k + 1) & 63);
    double beta, tkv, scale;
    if (ss == 0.0) {   // already reduced: no reflection
      tkv = 0.0;
      beta = x0;
      scale = 0.0;
    } else {
      const double nrm = sqrt(x0 * x0 + ss);
      beta = x0 >= 0.0 ? -nrm : nrm;
      tkv = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    double* vb = sv + 256 * (k & 1);
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int i = lane + 64 * s;
      const double vi = i == k + 1 ? 1.0 : (i > k + 1 && i < n ? x[s] * scale : 0.0);
      vb[i] = vi;
      if (i > k && i < n) refl[(int64_t)k * n + (i - k - 1)] = vi;
    }
    if (lane == 0) {
      s_tau[k & 1] = tkv;
      tau[k] = tkv;
      e[k] = beta;
      d[k] = dk;
    }
  };
  // step k = 8 T + w (w = k mod 8, a runtime value; T and the first row slot that can hold a row below k
  // (SLO = T / 8) fixed at compile time, so that no register is chosen at run time).  The
  // products run over all column slots from T on, with no tests: v and p are zero at the columns j <= k and
  // j >= n and at the rows i <= k, so those elements take exact zero updates (also when tau = 0, which makes
  // p and w zero)
  auto step = [&](int k, int w, auto Tc) {
    constexpr int T = decltype(Tc)::value, SLO = T / 8;   // rows in slots below SLO are at or above k
    const double* vb = sv + 256 * (k & 1);
    const double tk = s_tau[k & 1];
    // v at this wave's columns, slot t in lane t mod 16 of every row of 16 lanes (of vc0 for t < 16, of vc1
    // above), handed to all lanes by row broadcasts
    const int c16 = wave + 8 * (lane & 15);
    const double vc0 = vb[c16], vc1 = vb[c16 + 128];
    auto colv = [&](auto tc, double x0, double x1) {
      constexpr int t = decltype(tc)::value;
      if constexpr (t < 16)
        return row_bcast<t>(x0);
      else
        return row_bcast<(t >= 16 ? t - 16 : 0)>(x1);
    };
    // p partials: r_s = sum over this thread's columns of A(i, j) v_j
    double r[RS];
#pragma unroll
    for (int s = SLO; s < RS; ++s) r[s] = 0.0;
    static_for<T, CS>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      const double vj = colv(tc, vc0, vc1);
#pragma unroll
      for (int s = SLO; s < RS; ++s) r[s] = fma(a[s][t], vj, r[s]);
      __builtin_amdgcn_sched_barrier(0);   // each broadcast next to its use (not all hoisted into registers)
    });
#pragma unroll
    for (int s = SLO; s < RS; ++s) sPr[wave * 256 + lane + 64 * s] = r[s];
    lds_barrier();
    if (tid < 64 * RS) {
      const int i = tid;
      double p = 0.0;
      if (i > k && i < n) {
        const double* q = sPr + i;
        p = tk * (((q[0] + q[256]) + (q[512] + q[768])) + ((q[1024] + q[1280]) + (q[1536] + q[1792])));
      }
      sp[i] = p;
    }
    lds_barrier();
    // -v and -w at this thread's rows (held negated, so that the update is two plain FMAs)
    double nv[RS], nw[RS], dot = 0.0;
#pragma unroll
    for (int s = SLO; s < RS; ++s) {
      nv[s] = -vb[lane + 64 * s];
      nw[s] = -sp[lane + 64 * s];
      dot = fma(nw[s], nv[s], dot);
    }
    const double K = 0.5 * tk * wave_sum64(dot);
#pragma unroll
    for (int s = SLO; s < RS; ++s) nw[s] = fma(-K, nv[s], nw[s]);
    const double wc0 = fma(-K, vc0, sp[c16]), wc1 = fma(-K, vc1, sp[c16 + 128]);
    // A -= v w^T + w v^T on this thread's elements, as two rounded FMAs per element
    auto updated = [&](int s, double aij, double vj, double wj) { return fma(nw[s], vj, fma(nv[s], wj, aij)); };
    static_for<T, CS>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      const double vj = colv(tc, vc0, vc1), wj = colv(tc, wc0, wc1);
#pragma unroll
      for (int s = SLO; s < RS; ++s) {
        a[s][t] = updated(s, a[s][t], vj, wj);
        asm volatile("" : "+v"(a[s][t]));   // updated here, not sunk to later uses with the broadcasts held live
      }
    });
    // reflector k+1 from the updated column k+1, in slot T, or T + 1 after the last step of the group (a
    // branch that only reads the tile)
    if (k + 1 < n - 2 && wave == ((w + 1) & 7)) {
      double x[RS];
      if (w < 7) {
#pragma unroll
        for (int s = 0; s < RS; ++s) x[s] = a[s][T];
        reflector(k + 1, x);
      } else if constexpr (T + 1 < CS) {
#pragma unroll
        for (int s = 0; s < RS; ++s) x[s] = a[s][T + 1];
        reflector(k + 1, x);
      }
    }
    if (k == n - 3) {   // the last 2 x 2 block: columns n-2 and n-1, in slot T or T+1
      static_for<T, (T + 2 < CS ? T + 2 : CS)>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
#pragma unroll
        for (int s = SLO; s < RS; ++s) {
          const int i = lane + 64 * s, j = wave + 8 * t;
          if (i == j && i >= n - 2 && i < n) d[i] = a[s][t];
          if (i == n - 1 && j == n - 2) e[n - 2] = a[s][t];
        }
      });
    }
  };
  if (wave == 0) {
    double x[RS];
#pragma unroll
    for (int s = 0; s < RS; ++s) x[s] = a[s][0];
    reflector(0, x);
  }
  // the eight steps of a group in one loop (a second copy of the step would hold a second register tile at
  // the join)
  static_for<0, CS>([&](auto Tc) {
    constexpr int T = decltype(Tc)::value;
    for (int w = 0; w < 8; ++w) {
      const int k = 8 * T + w;
      if (k >= n - 2) break;   // uniform
      lds_barrier();           // v_k and tau_k
      step(k, w, std::integral_constant<int, T>{});
    }
  });
  if (tid == 0) {
    e[n - 1] = 0.0;
    tau[n - 2] = 0.0;
    tau[n - 1] = 0.0;
  }
}

// launch k_tridiag_reg for matrices of order up to nmax (at most kTriRegMax)
static void launch_tridiag_reg(const double* A, int lda, int64_t strideA, const TriSizes& sz, int nmax, int count,
                               double* refl, double* tau, double* d, double* e, double* flag, hipStream_t s) {
  const size_t lds = tridiag_reg_lds_bytes();
#define RW_TRI_REG(RS, CS)                                                                                     \
  k_tridiag_reg<RS, CS><<<count, kTriRegThreads, lds, s>>>(A, lda, strideA, sz, nmax, refl, tau, d, e, flag)
  if (nmax <= 64)
    RW_TRI_REG(1, 8);
  else if (nmax <= 128)
    RW_TRI_REG(2, 16);
  else if (nmax <= 192)
    RW_TRI_REG(3, 24);
  else if (nmax <= 200)
    RW_TRI_REG(4, 25);
  else
    RW_TRI_REG(4, 28);
#undef RW_TRI_REG
}

// Sturm count: the number of eigenvalues of T below sigma (the negative pivots of LDL^T of T - sigma I,
// a pivot of magnitude below pivmin taken as -pivmin)
// 1 / q from the hardware reciprocal and two Newton steps (a few units in the last place; |q| >= pivmin, a
// normal number, keeps it finite)
__device__ __forceinline__ double tr_recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}
// the Sturm count's 1 / q with one Newton step (about 11 ulp, measured): the computed count is then the
// exact count of T with each e^2 perturbed by some ten units in the last place, which moves an eigenvalue
// by about 10 u |T| (a few times the multisection's stopping width 4 u |T|); each step's dependent chain
// is two operations shorter than with two Newton steps
__device__ __forceinline__ double tr_recip1(double q) {
  const double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}

// (the operands of eight steps are loaded before their chain, so that a step waits for arithmetic only)
__device__ __forceinline__ int tr_sturm(const double* d, const double* e2, int n, double sigma, double pivmin) {
  double q = d[0] - sigma;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  int j = 1;
  for (; j + 8 <= n; j += 8) {
    double dv[8], ev[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      dv[u] = d[j + u];
      ev[u] = e2[j + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      q = (dv[u] - sigma) - ev[u] * tr_recip1(q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
  }
  for (; j < n; ++j) {
    q = (d[j] - sigma) - e2[j - 1] * tr_recip1(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// 2. eigenvalue idx = blockIdx.x (ascending) by multisection: each pass evaluates Sturm counts at
// kBisThreads interior points of [a, b] (one per thread) and keeps the subinterval where the count passes
// idx (the interval shrinks (kBisThreads + 1)-fold per pass)
constexpr int kBisThreads = 256;
__global__ __launch_bounds__(kBisThreads) void k_tri_bisect(const double* dg, const double* eg, TriSizes sz,
                                                            int nmax, double* lam, double* flag) {
  __shared__ double d[256], e2[256];
  __shared__ int s_cnt[2][kBisThreads / 64];
  const int idx = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = sz.n[blockIdx.y];
  if (idx >= n) return;   // the whole workgroup
  dg += (int64_t)blockIdx.y * nmax;
  eg += (int64_t)blockIdx.y * nmax;
  lam += (int64_t)blockIdx.y * nmax;
  // Gershgorin bounds, in every wave (identical results)
  double lo = INFINITY, hi = -INFINITY, tn = 0.0, emax = 0.0;
  for (int j = lane; j < n; j += 64) {
    const double el = j > 0 ? fabs(eg[j - 1]) : 0.0, er = j < n - 1 ? fabs(eg[j]) : 0.0;
    if (wave == 0) {
      d[j] = dg[j];
      if (j < n - 1) e2[j] = eg[j] * eg[j];
    }
    lo = fmin(lo, dg[j] - el - er);
    hi = fmax(hi, dg[j] + el + er);
    tn = fmax(tn, fabs(dg[j]) + el + er);
    emax = fmax(emax, er * er);
  }
  lo = wave_min64(lo);
  hi = wave_max64(hi);
  tn = wave_max64(tn);
  emax = wave_max64(emax);
  __syncthreads();
  const double pivmin = 2.3e-308 * fmax(1.0, emax);
  const double atol = 4.0 * 2.3e-16 * fmax(tn, 1e-300);
  constexpr double kParts = kBisThreads + 1;
  double a = lo - atol, b = hi + atol;   // count(a) <= idx < count(b); a, b identical in every thread
  for (int it = 0; it < 16 && b - a > atol; ++it) {
    const double sigma = a + (b - a) * (double)(tid + 1) / kParts;
    const int cnt = tr_sturm(d, e2, n, sigma, pivmin);
    const unsigned long long le = __ballot(cnt <= idx);   // counts grow with sigma: threads 0..L-1
    if (lane == 0) s_cnt[it & 1][wave] = __popcll(le);
    __syncthreads();
    int L = 0;
#pragma unroll
    for (int w = 0; w < kBisThreads / 64; ++w) L += s_cnt[it & 1][w];
    const double na = L > 0 ? a + (b - a) * (double)L / kParts : a;
    const double nb = L < kBisThreads ? a + (b - a) * (double)(L + 1) / kParts : b;
    a = na;
    b = nb;
  }
  const double lam_i = 0.5 * (a + b);
  if (tid == 0) lam[idx] = lam_i;
}

// 3. inverse iteration: eigenvector i = global thread index, three solves with LDL^T of T - lambda_i I
// (pivots of magnitude below pivmin replaced by pivmin with their sign).  A workgroup of kInvitThreads
// threads (32, or 16 where 32 vectors do not fit in LDS) keeps T, its threads' factors (L_j and 1 / D_j)
// and iterates in LDS, entry j of thread t at j * kInvitThreads + t; Z(j, i) is written at j * n + i.
constexpr int kInvB = 8;   // rows of a recurrence staged in registers at a time
static size_t invit_lds_bytes(int n, int tpb) { return ((size_t)n * (2 + 3 * tpb)) * sizeof(double); }
static int invit_threads(int n) { return invit_lds_bytes(n, 32) <= kLdsLimit ? 32 : 16; }

template <int kInvitThreads>
__global__ __launch_bounds__(kInvitThreads) void k_tri_invit(const double* dg, const double* eg, TriSizes sz,
                                                             int nmax, const double* lam, double* Z) {
  const int n = sz.n[blockIdx.y];
  if ((int)blockIdx.x * kInvitThreads >= n) return;   // the whole workgroup
  dg += (int64_t)blockIdx.y * nmax;
  eg += (int64_t)blockIdx.y * nmax;
  lam += (int64_t)blockIdx.y * nmax;
  Z += (int64_t)blockIdx.y * nmax * nmax;
  extern __shared__ double sm[];
  double* d = sm;
  double* e = d + n;
  double* Lf = e + n;
  double* rD = Lf + (size_t)n * kInvitThreads;
  double* z = rD + (size_t)n * kInvitThreads;
  const int t = threadIdx.x, i = blockIdx.x * kInvitThreads + t;
  double tn = 0.0;
  for (int j = t; j < n; j += kInvitThreads) {
    d[j] = dg[j];
    e[j] = eg[j];
    tn = fmax(tn, fabs(dg[j]) + (j > 0 ? fabs(eg[j - 1]) : 0.0) + (j < n - 1 ? fabs(eg[j]) : 0.0));
  }
  for (int o = kInvitThreads / 2; o > 0; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o, kInvitThreads));
  __syncthreads();
  if (i >= n) return;
  const double pivmin = 2.3e-16 * fmax(tn, 1e-290);   // a normal number (tr_recip)
  const double l = lam[i];
  // Each recurrence below runs over whole blocks of kInvB rows whose operands are loaded into registers
  // first and whose results are stored after (a step then waits for arithmetic, not for an LDS round trip),
  // and over the remaining rows one at a time.
  // factor: D_0 = d_0 - l, L_j = e_{j-1} / D_{j-1}, D_j = d_j - l - L_j e_{j-1}
  // (the reciprocals by tr_recip: a few ulp, a perturbation of the factors the iteration does not notice)
  double D = d[0] - l;
  if (fabs(D) < pivmin) D = D < 0.0 ? -pivmin : pivmin;
  double r = tr_recip(D);
  rD[t] = r;
  int j = 1;
  for (; j + kInvB <= n; j += kInvB) {
    double dv[kInvB], ev[kInvB], Lv[kInvB], rv[kInvB];
#pragma unroll
    for (int u = 0; u < kInvB; ++u) {
      dv[u] = d[j + u];
      ev[u] = e[j + u - 1];
    }
#pragma unroll
    for (int u = 0; u < kInvB; ++u) {
      const double Lj = ev[u] * r;
      double Dj = (dv[u] - l) - Lj * ev[u];
      if (fabs(Dj) < pivmin) Dj = Dj < 0.0 ? -pivmin : pivmin;
      r = tr_recip(Dj);
      Lv[u] = Lj;
      rv[u] = r;
    }
#pragma unroll
    for (int u = 0; u < kInvB; ++u) {
      Lf[(j + u) * kInvitThreads + t] = Lv[u];
      rD[(j + u) * kInvitThreads + t] = rv[u];
    }
  }
  for (; j < n; ++j) {
    const double Lj = e[j - 1] * r;
    double Dj = (d[j] - l) - Lj * e[j - 1];
    if (fabs(Dj) < pivmin) Dj = Dj < 0.0 ? -pivmin : pivmin;
    r = tr_recip(Dj);
    Lf[j * kInvitThreads + t] = Lj;
    rD[j * kInvitThreads + t] = r;
  }
  // start vector: deterministic, with no special structure: 1 + sin(0.7 j + 1.3 i + 0.1) / 2, the sines by
  // the three-term recurrence s_{j+1} = 2 cos(0.7) s_j - s_{j-1} (n >= 3)
  {
    const double c2 = 2.0 * cos(0.7);
    double s0 = sin(1.3 * i + 0.1), s1 = sin(0.7 + 1.3 * i + 0.1);
    z[t] = 1.0 + 0.5 * s0;
    z[kInvitThreads + t] = 1.0 + 0.5 * s1;
    for (int jj = 2; jj < n; ++jj) {
      const double s2 = c2 * s1 - s0;
      z[jj * kInvitThreads + t] = 1.0 + 0.5 * s2;
      s0 = s1;
      s1 = s2;
    }
  }
  double inv = 1.0;   // the previous iteration's 1 / ||x||, applied as b is read
  for (int it = 0; it < 3; ++it) {
    // forward: y_j = b_j - L_j y_{j-1}
    double y = z[t] * inv;
    z[t] = y;
    j = 1;
    for (; j + kInvB <= n; j += kInvB) {
      double zv[kInvB], lv[kInvB];
#pragma unroll
      for (int u = 0; u < kInvB; ++u) {
        zv[u] = z[(j + u) * kInvitThreads + t] * inv;
        lv[u] = Lf[(j + u) * kInvitThreads + t];
      }
#pragma unroll
      for (int u = 0; u < kInvB; ++u) {
        y = zv[u] - lv[u] * y;
        zv[u] = y;
      }
#pragma unroll
      for (int u = 0; u < kInvB; ++u) z[(j + u) * kInvitThreads + t] = zv[u];
    }
    for (; j < n; ++j) {
      y = z[j * kInvitThreads + t] * inv - Lf[j * kInvitThreads + t] * y;
      z[j * kInvitThreads + t] = y;
    }
    // backward: x_{n-1} = y_{n-1} / D_{n-1}, x_j = y_j / D_j - L_{j+1} x_{j+1}
    double x = y * rD[(n - 1) * kInvitThreads + t];
    z[(n - 1) * kInvitThreads + t] = x;
    double nrm = x * x;
    j = n - 2;
    for (; j - kInvB + 1 >= 0; j -= kInvB) {
      double zv[kInvB], rv[kInvB], lv[kInvB];
#pragma unroll
      for (int u = 0; u < kInvB; ++u) {
        zv[u] = z[(j - u) * kInvitThreads + t];
        rv[u] = rD[(j - u) * kInvitThreads + t];
        lv[u] = Lf[(j - u + 1) * kInvitThreads + t];
      }
#pragma unroll
      for (int u = 0; u < kInvB; ++u) {
        x = zv[u] * rv[u] - lv[u] * x;
        zv[u] = x;
        nrm += x * x;
      }
#pragma unroll
      for (int u = 0; u < kInvB; ++u) z[(j - u) * kInvitThreads + t] = zv[u];
    }
    for (; j >= 0; --j) {
      x = z[j * kInvitThreads + t] * rD[j * kInvitThreads + t] - Lf[(j + 1) * kInvitThreads + t] * x;
      z[j * kInvitThreads + t] = x;
      nrm += x * x;
    }
    inv = 1.0 / sqrt(nrm);
  }
  for (int jj = 0; jj < n; ++jj) Z[(int64_t)jj * n + i] = z[jj * kInvitThreads + t] * inv;
}

// 3b. clusters.  One wave per matrix walks the eigenvalues in order; for a cluster (successive
// eigenvalues closer than kClusterRel |T|) the first vector is kept and each later one is computed again
// from its own inverse-iteration vector: LDL^T of T - lambda I (lane 0), then three times Gram-Schmidt
// against the cluster's earlier vectors (twice, all lanes), normalization and one solve, and a final
// Gram-Schmidt and normalization.  The cluster's vectors are held in LDS (at most kTriClusterMax).
// flag[0] = 1 for a longer cluster, or when a vector vanishes under the orthogonalization.
constexpr double kClusterRel = 1e-6;
constexpr int kTriClusterMax = 32;
static size_t cluster_lds_bytes(int nmax) { return ((size_t)kTriClusterMax + 5) * nmax * sizeof(double); }

__global__ __launch_bounds__(64) void k_tri_cluster(const double* dg, const double* eg, TriSizes sz, int nmax,
                                                    const double* lam, double* Z, double* flag) {
  const int b = blockIdx.x, n = sz.n[b], lane = threadIdx.x;
  dg += (int64_t)b * nmax;
  eg += (int64_t)b * nmax;
  lam += (int64_t)b * nmax;
  Z += (int64_t)b * nmax * nmax;   // Z(j, i) at j * n + i
  extern __shared__ double sm[];
  double* d = sm;
  double* e = d + nmax;
  double* Lf = e + nmax;
  double* rD = Lf + nmax;
  double* x = rD + nmax;
  double* cl = x + nmax;   // cluster vectors, vector c at c * nmax
  double tn = 0.0;
  for (int j = lane; j < n; j += 64) {
    d[j] = dg[j];
    e[j] = eg[j];
    tn = fmax(tn, fabs(dg[j]) + (j > 0 ? fabs(eg[j - 1]) : 0.0) + (j < n - 1 ? fabs(eg[j]) : 0.0));
  }
  tn = wave_max64(tn);
  __syncthreads();
  const double thr = kClusterRel * tn;
  const double pivmin = 2.3e-16 * fmax(tn, 1e-290);
  auto dot = [&](const double* u, const double* v) -> double {
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += u[j] * v[j];
    return wave_sum64(s);
  };
  int i = 1;
  while (i < n) {   // uniform: every lane reads the same eigenvalues
    if (!(lam[i] - lam[i - 1] < thr)) {
      ++i;
      continue;
    }
    const int c0 = i - 1;
    int c1 = i;
    while (c1 + 1 < n && lam[c1 + 1] - lam[c1] < thr) ++c1;
    if (c1 - c0 + 1 > kTriClusterMax) {
      if (lane == 0) flag[0] = 1.0;
      return;
    }
    for (int j = lane; j < n; j += 64) cl[j] = Z[(int64_t)j * n + c0];
    for (int v = c0 + 1; v <= c1; ++v) {
      const int nv = v - c0;   // earlier vectors of the cluster in cl[0 .. nv)
      for (int j = lane; j < n; j += 64) x[j] = Z[(int64_t)j * n + v];
      const double l = lam[v];
      if (lane == 0) {   // LDL^T of T - l I
        double D = d[0] - l;
        if (fabs(D) < pivmin) D = D < 0.0 ? -pivmin : pivmin;
        double r = 1.0 / D;
        rD[0] = r;
        for (int j = 1; j < n; ++j) {
          const double Lj = e[j - 1] * r;
          double Dj = (d[j] - l) - Lj * e[j - 1];
          if (fabs(Dj) < pivmin) Dj = Dj < 0.0 ? -pivmin : pivmin;
          r = 1.0 / Dj;
          Lf[j] = Lj;
          rD[j] = r;
        }
      }
      __syncthreads();
      auto orth_normalize = [&]() -> double {
        for (int pass = 0; pass < 2; ++pass)
          for (int c = 0; c < nv; ++c) {
            const double h = dot(cl + (int64_t)c * nmax, x);
            for (int j = lane; j < n; j += 64) x[j] -= h * cl[(int64_t)c * nmax + j];
            __syncthreads();
          }
        const double nrm = sqrt(dot(x, x));
        const double s = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int j = lane; j < n; j += 64) x[j] *= s;
        __syncthreads();
        return nrm;
      };
      double nrm = orth_normalize();
      for (int it = 0; it < 3; ++it) {
        if (lane == 0) {   // solve L D L^T y = x in place
          double y = x[0];
          for (int j = 1; j < n; ++j) {
            y = x[j] - Lf[j] * y;
            x[j] = y;
          }
          double xx = y * rD[n - 1];
          x[n - 1] = xx;
          for (int j = n - 2; j >= 0; --j) {
            xx = x[j] * rD[j] - Lf[j + 1] * xx;
            x[j] = xx;
          }
        }
        __syncthreads();
        nrm = orth_normalize();
      }
      if (!(nrm > 0.0) || !isfinite(nrm)) {
        if (lane == 0) flag[0] = 1.0;
        return;
      }
      for (int j = lane; j < n; j += 64) {
        cl[(int64_t)nv * nmax + j] = x[j];
        Z[(int64_t)j * n + v] = x[j];
      }
      __syncthreads();
    }
    i = c1 + 1;
  }
}

constexpr int kTriAhead = 16;   // reflectors loaded ahead by the back-transform and the right-hand-side pass

// 4. V(:, col) = H_0 H_1 ... H_{n-3} z, z = eigenvector col of T; V column-major n x n
__global__ __launch_bounds__(64) void k_tri_back(const double* refl, const double* tau, int n, const double* Z,
                                                 double* V) {
  const int col = blockIdx.x, lane = threadIdx.x;
  double z[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = lane + 64 * q;
    z[q] = r < n ? Z[(int64_t)r * n + col] : 0.0;
  }
  // reflector k's entries for this lane's rows, loaded one step ahead
  auto fetch = [&](int k, double (&vr)[4]) {
    const double* vk = refl + (int64_t)k * n;
    const int m = n - k - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q - (k + 1);
      vr[q] = (k >= 0 && i >= 0 && i < m) ? vk[i] : 0.0;
    }
  };
  // reflectors k, k-1, .., k-kTriAhead+1 in flight (written on another XCD, so most loads miss this L2)
  double vb[kTriAhead][4], tb[kTriAhead];
#pragma unroll
  for (int u = 0; u < kTriAhead; ++u) {
    fetch(n - 3 - u, vb[u]);
    tb[u] = n - 3 - u >= 0 ? tau[n - 3 - u] : 0.0;
  }
  for (int k0 = n - 3; k0 >= 0; k0 -= kTriAhead) {
#pragma unroll
    for (int u = 0; u < kTriAhead; ++u) {
      const int k = k0 - u;
      if (k < 0) break;
      const double tk = tb[u];
      if (tk != 0.0) {   // uniform
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) s += vb[u][q] * z[q];
        s = tr_wave_sum(s) * tk;
#pragma unroll
        for (int q = 0; q < 4; ++q) z[q] -= s * vb[u][q];
      }
      fetch(k - kTriAhead, vb[u]);
      tb[u] = k - kTriAhead >= 0 ? tau[k - kTriAhead] : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = lane + 64 * q;
    if (r < n) V[r + (int64_t)col * n] = z[q];
  }
}


// 5. (right-hand sides) h = U^T r = H_{n-3} ... H_1 H_0 r for right-hand side c = blockIdx.x of matrix
// blockIdx.y (r: column c of R, ld ldr, matrices strideR apart; h: nmax x C per matrix), one wave each
__global__ __launch_bounds__(64) void k_tri_rhs(const double* refl, const double* tau, TriSizes sz, int nmax,
                                                const double* R, int ldr, int64_t strideR, int C, double* h) {
  const int c = blockIdx.x, b = blockIdx.y, lane = threadIdx.x, n = sz.n[b];
  refl += (int64_t)b * nmax * nmax;
  tau += (int64_t)b * nmax;
  const double* r = R + b * strideR + (int64_t)c * ldr;
  double z[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    z[q] = i < n ? r[i] : 0.0;
  }
  auto fetch = [&](int k, double (&vr)[4]) {
    const double* vk = refl + (int64_t)k * n;
    const int m = n - k - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q - (k + 1);
      vr[q] = (k <= n - 3 && i >= 0 && i < m) ? vk[i] : 0.0;
    }
  };
  double vb[kTriAhead][4], tb[kTriAhead];
#pragma unroll
  for (int u = 0; u < kTriAhead; ++u) {
    fetch(u, vb[u]);
    tb[u] = u <= n - 3 ? tau[u] : 0.0;
  }
  for (int k0 = 0; k0 <= n - 3; k0 += kTriAhead) {
#pragma unroll
    for (int u = 0; u < kTriAhead; ++u) {
      const int k = k0 + u;
      if (k > n - 3) break;
      const double tk = tb[u];
      if (tk != 0.0) {   // uniform
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) t += vb[u][q] * z[q];
        t = tr_wave_sum(t) * tk;
#pragma unroll
        for (int q = 0; q < 4; ++q) z[q] -= t * vb[u][q];
      }
      fetch(k + kTriAhead, vb[u]);
      tb[u] = k + kTriAhead <= n - 3 ? tau[k + kTriAhead] : 0.0;
    }
  }
  double* hc = h + ((int64_t)b * C + c) * nmax;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    if (i < n) hc[i] = z[q];
  }
}

// 6. (right-hand sides) w_i = lambda_i and R(i, c) = (Z^T h_c)_i for i < n, zero for n <= i < ldr; one wave
// per (i, matrix).  Nothing is written when the cluster flag is set (the caller falls back with R intact).
__global__ __launch_bounds__(64) void k_tri_rot(const double* Z, const double* lam, const double* h, TriSizes sz,
                                                int nmax, int C, const double* flag, double* w, double* R, int ldr,
                                                int64_t strideR) {
  if (flag[0] != 0.0) return;
  const int i = blockIdx.x, b = blockIdx.y, lane = threadIdx.x, n = sz.n[b];
  double* rb = R + b * strideR;
  if (i >= n) {
    for (int c = lane; c < C; c += 64) rb[(int64_t)c * ldr + i] = 0.0;
    if (lane == 0) w[(int64_t)b * ldr + i] = 0.0;
    return;
  }
  const double* Zb = Z + (int64_t)b * nmax * nmax;   // Z(j, i) at j * n + i
  for (int c = 0; c < C; ++c) {
    const double* hc = h + ((int64_t)b * C + c) * nmax;
    double t = 0.0;
    for (int j = lane; j < n; j += 64) t += Zb[(int64_t)j * n + i] * hc[j];
    t = tr_wave_sum(t);
    if (lane == 0) rb[(int64_t)c * ldr + i] = t;
  }
  if (lane == 0) w[(int64_t)b * ldr + i] = lam[(int64_t)b * nmax + i];
}

static void tri_attrs() {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_tridiag), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kLdsLimit);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_tri_invit<32>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_tri_invit<16>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_tri_cluster),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
    const void* reg[] = {reinterpret_cast<const void*>(k_tridiag_reg<1, 8>),
                         reinterpret_cast<const void*>(k_tridiag_reg<2, 16>),
                         reinterpret_cast<const void*>(k_tridiag_reg<3, 24>),
                         reinterpret_cast<const void*>(k_tridiag_reg<4, 25>),
                         reinterpret_cast<const void*>(k_tridiag_reg<4, 28>)};
    for (const void* f : reg)
      (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tridiag_reg_lds_bytes());
    attr = true;
  }
}

static void launch_invit(const double* d, const double* e, const TriSizes& sz, int nmax, int count, const double* lam,
                         double* Z, hipStream_t s) {
  if (invit_threads(nmax) == 32)
    k_tri_invit<32><<<dim3((nmax + 31) / 32, count), 32, invit_lds_bytes(nmax, 32), s>>>(d, e, sz, nmax, lam, Z);
  else
    k_tri_invit<16><<<dim3((nmax + 15) / 16, count), 16, invit_lds_bytes(nmax, 16), s>>>(d, e, sz, nmax, lam, Z);
}

size_t tridiag_rhs_work_count(int nmax, int count, int C) {
  return (size_t)count * (2 * (size_t)nmax * nmax + (size_t)(4 + C) * nmax) + 8;
}

int syev_tridiag_rhs(const double* A, int ld, const int* sizes, int count, double* R, int C, double* w, double* work,
                     size_t work_count, hipStream_t s, const double** flag_dev) {
  RW_CHECK(count >= 1 && count <= kTriBatchMax && C >= 1, RW_EINVAL, "batched tridiagonal solver: bad batch");
  TriSizes sz;
  int nmax = 0;
  for (int b = 0; b < count; ++b) {
    RW_CHECK(tridiag_batch_fits(sizes[b]) && sizes[b] <= ld, RW_EINVAL, "batched tridiagonal solver: n = %d",
             sizes[b]);
    sz.n[b] = sizes[b];
    nmax = std::max(nmax, sizes[b]);
  }
  RW_CHECK(work_count >= tridiag_rhs_work_count(nmax, count, C), RW_EWORKSPACE, "batched tridiagonal solver: "
           "workspace too small");
  const size_t nn = (size_t)nmax * nmax;
  double* refl = work;
  double* Z = refl + count * nn;
  double* tau = Z + count * nn;
  double* d = tau + (size_t)count * nmax;
  double* e = d + (size_t)count * nmax;
  double* lam = e + (size_t)count * nmax;
  double* h = lam + (size_t)count * nmax;
  double* flag = h + (size_t)count * nmax * C;
  tri_attrs();
  const int64_t strideR = (int64_t)ld * C;
  launch_tridiag_reg(A, ld, (int64_t)ld * ld, sz, nmax, count, refl, tau, d, e, flag, s);
  k_tri_rhs<<<dim3(C, count), 64, 0, s>>>(refl, tau, sz, nmax, R, ld, strideR, C, h);
  k_tri_bisect<<<dim3(nmax, count), kBisThreads, 0, s>>>(d, e, sz, nmax, lam, flag);
  launch_invit(d, e, sz, nmax, count, lam, Z, s);
  k_tri_cluster<<<count, 64, cluster_lds_bytes(nmax), s>>>(d, e, sz, nmax, lam, Z, flag);
  k_tri_rot<<<dim3(ld, count), 64, 0, s>>>(Z, lam, h, sz, nmax, C, flag, w, R, ld, strideR);
  RW_LAUNCH_CHECK();
  if (flag_dev != nullptr) {
    *flag_dev = flag;
    return RW_OK;
  }
  double fl = 0.0;
  RW_HIP(hipMemcpyAsync(&fl, flag, sizeof(double), hipMemcpyDeviceToHost, s));
  RW_HIP(hipStreamSynchronize(s));
  return fl != 0.0 ? RW_ENOCONV : RW_OK;
}

int syev_tridiag(const double* A, double* w, double* V, int n, double* work, hipStream_t s, const double** flag_dev) {
  RW_CHECK(tridiag_fits(n), RW_EINVAL, "tridiagonal eigensolver: n = %d out of range", n);
  const TriBufs b = tri_bufs(work, n);
  tri_attrs();
  TriSizes sz;
  sz.n[0] = n;
  // orders up to kTriRegMax: the matrix in registers; above: the first n - kTriLdsMax columns on a full copy in
  // b.Lf (n x n, unused otherwise), the rest packed in LDS
  if (n <= kTriRegMax) {
    launch_tridiag_reg(A, n, 0, sz, n, 1, b.refl, b.tau, b.d, b.e, b.flag, s);
  } else {
    const int nl = std::min(n, kTriLdsMax);
    k_tridiag<<<1, 1024, tridiag_lds_bytes(nl), s>>>(A, n, 0, sz, n, b.refl, b.tau, b.d, b.e, b.flag, b.Lf, n - nl);
  }
  // the eigenvalues go straight to w (bisection, inverse iteration and the cluster pass read them there)
  k_tri_bisect<<<n, kBisThreads, 0, s>>>(b.d, b.e, sz, n, w, b.flag);
  launch_invit(b.d, b.e, sz, n, 1, w, b.Z, s);
  k_tri_cluster<<<1, 64, cluster_lds_bytes(n), s>>>(b.d, b.e, sz, n, w, b.Z, b.flag);
  k_tri_back<<<n, 64, 0, s>>>(b.refl, b.tau, n, b.Z, V);
  RW_LAUNCH_CHECK();
  if (flag_dev != nullptr) {
    *flag_dev = b.flag;
    return RW_OK;
  }
  double flag = 0.0;
  RW_HIP(hipMemcpyAsync(&flag, b.flag, sizeof(double), hipMemcpyDeviceToHost, s));
  RW_HIP(hipStreamSynchronize(s));
  if (flag != 0.0) return RW_ENOCONV;   // clustered eigenvalues: the caller uses the Jacobi solver
  return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_dense_syev_tridiag_workspace_bytes(int n, size_t* bytes) {
  RW_CHECK(bytes != nullptr && tridiag_fits(n), RW_EINVAL, "bad size n = %d", n);
  *bytes = tridiag_work_count(n) * sizeof(double);
  return RW_OK;
}

int rw_dense_syev_tridiag(const double* A, double* w, double* V, int n, void* work, size_t work_bytes,
                          hipStream_t stream) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(A != nullptr && w != nullptr && V != nullptr && work != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(tridiag_fits(n), RW_EINVAL, "tridiagonal eigensolver: n = %d out of range [3, 256]", n);
  RW_CHECK(work_bytes >= tridiag_work_count(n) * sizeof(double), RW_EWORKSPACE, "workspace too small");
  const int st = syev_tridiag(A, w, V, n, static_cast<double*>(work), stream);
  if (st == RW_ENOCONV) set_error("tridiagonal eigensolver: clustered eigenvalues (use the Jacobi routine)");
  return st;
}

int rw_dense_eig_rhs_batched_workspace_bytes(int nmax, int count, int nrhs, size_t* bytes) {
  RW_CHECK(bytes != nullptr && tridiag_batch_fits(nmax) && count >= 1 && count <= kTriBatchMax && nrhs >= 1, RW_EINVAL,
           "bad sizes (nmax = %d, count = %d, nrhs = %d)", nmax, count, nrhs);
  *bytes = tridiag_rhs_work_count(nmax, count, nrhs) * sizeof(double);
  return RW_OK;
}

int rw_dense_eig_rhs_batched(const double* A, int ld, const int* sizes, int count, double* R, int nrhs, double* w,
                             void* work, size_t work_bytes, hipStream_t stream) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(A != nullptr && sizes != nullptr && R != nullptr && w != nullptr && work != nullptr, RW_EINVAL,
           "null argument");
  const int st = syev_tridiag_rhs(A, ld, sizes, count, R, nrhs, w, static_cast<double*>(work),
                                  work_bytes / sizeof(double), stream);
  if (st == RW_ENOCONV) set_error("batched tridiagonal solver: clustered eigenvalues (use the Jacobi routine)");
  return st;
}

}  // extern "C"
