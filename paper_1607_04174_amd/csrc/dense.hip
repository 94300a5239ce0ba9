// Small dense FP64 kernels: Cholesky, triangular inverse, symmetric eigendecomposition (cyclic
// Jacobi) and LU with partial pivoting.  One workgroup owns one matrix held in global memory (it
// stays L2-resident at these sizes); batched launches give each matrix its own workgroup.
#include <cmath>

#include "jacobi_layout.h"
#include "rw_internal.h"

namespace rw {

// ---------------------------------------------------------------------------------------------
// Cholesky A = L L^T (lower, in place; the strict upper triangle is left untouched)
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_chol(double* As, int n, int* info) {
  double* A = As + (int64_t)blockIdx.x * n * n;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      double akk = A[k + k * n];
      if (!(akk > 0.0) || !isfinite(akk)) bad = k + 1;
      else A[k + k * n] = sqrt(akk);
    }
    __syncthreads();
    if (bad) break;
    const double piv = A[k + k * n];
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i + k * n] /= piv;
    __syncthreads();
    // trailing lower triangle: rows i >= j > k
    for (int j = k + 1 + ty; j < n; j += 32) {
      const double ljk = A[j + k * n];
      for (int i = j + tx; i < n; i += 32) A[i + j * n] -= A[i + k * n] * ljk;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) info[blockIdx.x] = bad;
}

int chol_batched(double* A, int n, int count, int* info, hipStream_t s) {
  if (n <= 0 || count <= 0) return RW_OK;
  k_chol<<<count, 1024, 0, s>>>(A, n, info);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// Rinv = (L^T)^{-1}: one wave back-substitutes column j of the upper-triangular inverse; each step's
// dot product is a butterfly reduction, so every lane obtains every x_i.
__global__ __launch_bounds__(256) void k_upper_inverse(const double* L, double* Rinv, int n) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n) return;
  double* x = Rinv + (int64_t)j * n;
  for (int i = j + 1 + lane; i < n; i += 64) x[i] = 0.0;
  // R(i,k) = L(k,i) = L[k + i*n]
  const double xj = 1.0 / L[j + j * n];
  if (lane == 0) x[j] = xj;
  for (int i = j - 1; i >= 0; --i) {
    double acc = 0.0;
    for (int k = i + 1 + lane; k <= j; k += 64) acc += L[k + i * n] * (k == j ? xj : x[k]);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    // every lane holds the same xi and stores it, so a lane's later read of x[i] follows its own store
    x[i] = -acc / L[i + i * n];
  }
}

int chol_upper_inverse(const double* L, double* Rinv, int n, hipStream_t s) {
  if (n <= 0) return RW_OK;
  k_upper_inverse<<<(n + 3) / 4, 256, 0, s>>>(L, Rinv, n);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// Cholesky factor and its transposed inverse in one workgroup (n <= 224): W = (L^T)^{-1} (upper triangular,
// zero below) for A = L L^T, A given by its lower triangle.  info = k + 1 at the first pivot that is not
// positive and finite (W untouched up to order 200), else 0.
constexpr int kCholInvMaxN = 200;   // the packed factor plus n reciprocal roots within the LDS budget

// The factorization is right-looking with unscaled columns (Schur complements A(i,j) -= A(i,k) A(j,k) /
// A(k,k)), with the matrix in registers: 512 threads, thread (lane, wave) holds A(i, j) for the rows
// i = lane + 64 s (s < RS) and the columns j = wave + 8 t (t < CS), both triangles filled from the lower
// one.  Step k: the wave holding column k has put the column below the diagonal, u_i = A(i, k), in the
// packed factor in LDS (column k, with 1 / A(k,k) in its diagonal place); after one barrier every thread
// applies A(i, j) -= u_i m_j with m_j = u_j / A(k,k) (only the lower triangle is read later; the upper one
// is updated alongside), m_j handed to all lanes by row broadcasts, and the wave holding column k+1 checks
// its pivot and writes its column at once.  Steps k = 8 T + w with T unrolled at compile time (the column
// slots of a step and the row slots below k are then known without tests); entries at or left of column k
// and at or above row k take exact zero updates.
// Then W: with D = diag(L) and the unit lower factor M = L D^{-1} (M(i, k) = m_i of step k), L^{-1} =
// D^{-1} M^{-1}; Y = M^{-1} by forward substitution on all columns at once in the same registers (each wave
// its own columns: no barriers), and W(j, i) = Y(i, j) / L(i, i).
__device__ __forceinline__ int cw_lo(int i, int j, int n) { return j * n - ((j * (j - 1)) >> 1) + (i - j); }  // i >= j

// Above order 200 the packed factor does not fit in LDS (GM): the columns u go to W's strict lower triangle
// instead (read back by the forward substitution, one column ahead, and overwritten at the end, so that W's
// contents are undefined when info is not 0), with two LDS buffers for the step's column.
constexpr int kCholRegThreads = 512;
constexpr int kCholRegMaxN = 224;
static size_t chol_reg_lds_bytes(int n) {
  return (n <= kCholInvMaxN ? (size_t)n * (n + 1) / 2 + n : (size_t)2 * 256 + 2 * n) * sizeof(double);
}

template <int RS, int CS, bool GM>
__global__ __launch_bounds__(kCholRegThreads) void k_chol_inv_reg(const double* G, int n, double* W, int* info) {
  static_assert(RS >= 1 && RS <= 4 && 8 * CS <= 64 * RS && (!GM || RS == 4), "layout");
  extern __shared__ double sP[];   // packed lower (column-major): u below the diagonal, 1 / A(k,k) on it
  double* su = sP;                 // GM: u of the step, two buffers of 256
  double* sinv = sP + 512;         // GM: 1 / A(k, k)
  double* rd = GM ? sP + 512 + n : sP + n * (n + 1) / 2;   // 1 / sqrt(A(k, k)) = 1 / L(k, k)
  __shared__ int s_bad[2], s_n;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid == 0) s_n = n;
  double a[RS][CS];
#pragma unroll
  for (int s = 0; s < RS; ++s)
#pragma unroll
    for (int t = 0; t < CS; ++t) {
      const int i = lane + 64 * s, j = wave + 8 * t;
      const int hi = max(i, j), lo = min(i, j);   // the lower triangle's entry, one load with no branch
      a[s][t] = (i < n && j < n) ? G[hi + (int64_t)lo * n] : 0.0;
    }
  // entry (i, k) of the packed factor for rows below k (clamped to a valid place; the caller zeroes the rest)
  auto below = [&](int i, int k) {   // k <= n - 1; GM: i < 256
    if constexpr (GM)
      return su[256 * (k & 1) + i];
    else
      return sP[cw_lo(min(max(i, k + 1), n - 1), k, n)];
  };
  auto inv_of = [&](int k) {
    if constexpr (GM)
      return sinv[k];
    else
      return sP[cw_lo(k, k, n)];
  };
  // column k from slot TK (its diagonal in row slot k >> 6), by the wave holding it
  auto column = [&](int k, auto tkc) {
    constexpr int TK = decltype(tkc)::value;
    double xk = a[0][TK];
#pragma unroll
    for (int s = 1; s < RS; ++s) xk = s == (k >> 6) ? a[s][TK] : xk;
    const double dkk = lane_read(xk, k & 63);
    const bool bad = !(dkk > 0.0) || !isfinite(dkk);
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int i = lane + 64 * s;
      if constexpr (GM) {
        su[256 * (k & 1) + i] = (i > k && i < n) ? a[s][TK] : 0.0;
        if (i > k && i < n) W[i + (int64_t)k * n] = a[s][TK];
      } else {
        if (i > k && i < n) sP[cw_lo(i, k, n)] = a[s][TK];
      }
    }
    if (lane == 0) {
      if constexpr (GM)
        sinv[k] = 1.0 / dkk;
      else
        sP[cw_lo(k, k, n)] = 1.0 / dkk;
      s_bad[k & 1] = bad ? k + 1 : 0;
      rd[k] = bad ? 0.0 : 1.0 / sqrt(dkk);
    }
  };
  auto step = [&](int k, int w, auto Tc) {
    constexpr int T = decltype(Tc)::value, SLO = T / 8;   // rows in slots below SLO are at or above k
    const double inv = inv_of(k);
    double u[RS];
#pragma unroll
    for (int s = SLO; s < RS; ++s) {
      const int i = lane + 64 * s;
      const double v = below(i, k);
      u[s] = (i > k && i < n) ? v : 0.0;
    }
    const int c16 = wave + 8 * (lane & 15);
    const double v0 = below(c16, k), v1 = below(c16 + 128, k);
    const double mc0 = (c16 > k && c16 < n) ? v0 * inv : 0.0;
    const double mc1 = (c16 + 128 > k && c16 + 128 < n) ? v1 * inv : 0.0;
    static_for<T, CS>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      double mj;
      if constexpr (t < 16)
        mj = row_bcast<t>(mc0);
      else
        mj = row_bcast<(t >= 16 ? t - 16 : 0)>(mc1);
#pragma unroll
      for (int s = SLO; s < RS; ++s) {
        a[s][t] -= u[s] * mj;
        asm volatile("" : "+v"(a[s][t]));   // updated here, not sunk to later uses
      }
    });
    // column k+1 sits in slot T, or T + 1 after the last step of the group (a branch that only reads the tile)
    if (k + 1 < n && wave == ((w + 1) & 7)) {
      if (w < 7)
        column(k + 1, std::integral_constant<int, T>{});
      else if constexpr (T + 1 < CS)
        column(k + 1, std::integral_constant<int, T + 1>{});
    }
  };
  if (wave == 0) column(0, std::integral_constant<int, 0>{});
  // a pivot that is not positive and finite is recorded (the first one) and the steps run on to the end with
  // meaningless values, with no early exit (every index stays within the matrix either way): merging the
  // register tile at many exits would cost registers
  int bad = 0;
  static_for<0, CS>([&](auto Tc) {
    constexpr int T = decltype(Tc)::value;
    using TT = std::integral_constant<int, T>;
    for (int w = 0; w < 8; ++w) {   // one loop of the eight steps (a second copy of the step would hold a
      const int k = 8 * T + w;       // second register tile at the join)
      if (k >= n) return;   // uniform
      lds_barrier();        // column k in LDS, its pivot checked
      if (bad == 0) bad = s_bad[k & 1];
      step(k, w, TT{});
    }
  });
  if constexpr (GM) __threadfence_block();   // the columns in W, for every wave
  __syncthreads();
  if (bad) {
    if (tid == 0) info[0] = bad;
    return;
  }
  // GM: column k of M from W, loaded one step ahead
  double ln[RS];
  auto load_col = [&](int k) {
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int i = lane + 64 * s;
      ln[s] = W[min(max(i, k + 1), n - 1) + (int64_t)k * n];
    }
  };
  if constexpr (GM) load_col(0);
  // Y = M^{-1}: start from I; step k subtracts M(i, k) Y(k, :) from the rows below k, where row k (final by
  // then) is read from the lane holding it and only the columns j <= k (slots up to T) are nonzero
#pragma unroll
  for (int s = 0; s < RS; ++s)
#pragma unroll
    for (int t = 0; t < CS; ++t) a[s][t] = (lane + 64 * s == wave + 8 * t) ? 1.0 : 0.0;
  static_for<0, CS>([&](auto Tc) {
    constexpr int T = decltype(Tc)::value, SK = T / 8, SLO = T / 8;
    for (int w = 0; w < 8; ++w) {
      const int k = 8 * T + w;
      if (k >= n - 1) return;   // uniform
      const double inv = inv_of(k);
      double l[RS];
#pragma unroll
      for (int s = SLO; s < RS; ++s) {
        const int i = lane + 64 * s;
        double v;
        if constexpr (GM)
          v = ln[s];
        else
          v = below(i, k);
        l[s] = (i > k && i < n) ? v * inv : 0.0;
      }
      if constexpr (GM) {
        if (k + 1 < n - 1) load_col(k + 1);
      }
      static_for<0, T + 1>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        const double yk = lane_read(a[SK][t], k & 63);
#pragma unroll
        for (int s = SLO; s < RS; ++s) {
          a[s][t] -= l[s] * yk;
          asm volatile("" : "+v"(a[s][t]));
        }
      });
    }
  });
  // W(j, i) = Y(i, j) / L(i, i) on and above the diagonal, zero below (the order read back from LDS here, so
  // that these addresses are formed now and not held through the steps); GM: after every wave's last read
  // of W's lower triangle
  if constexpr (GM) __syncthreads();
  const int n2 = __builtin_amdgcn_readfirstlane(s_n);
#pragma unroll
  for (int s = 0; s < RS; ++s)
#pragma unroll
    for (int t = 0; t < CS; ++t) {
      const int i = lane + 64 * s, j = wave + 8 * t;
      if (i < n2 && j < n2) W[j + (int64_t)i * n2] = i >= j ? a[s][t] * rd[i] : 0.0;
    }
  if (tid == 0) info[0] = 0;
}

int chol_inverse(double* G, double* W, int n, int* info, hipStream_t s) {
  if (n <= 0) return RW_OK;
  if (n > kCholRegMaxN) {
    RW_TRY(chol_batched(G, n, 1, info, s));
    int bad = 0;
    RW_HIP(hipMemcpyAsync(&bad, info, sizeof(int), hipMemcpyDeviceToHost, s));
    RW_HIP(hipStreamSynchronize(s));
    if (bad == 0) RW_TRY(chol_upper_inverse(G, W, n, s));
    return RW_OK;
  }
  static bool attr = false;
  if (!attr) {
    const void* ks[] = {reinterpret_cast<const void*>(k_chol_inv_reg<1, 8, false>),
                        reinterpret_cast<const void*>(k_chol_inv_reg<2, 16, false>),
                        reinterpret_cast<const void*>(k_chol_inv_reg<3, 24, false>),
                        reinterpret_cast<const void*>(k_chol_inv_reg<4, 25, false>),
                        reinterpret_cast<const void*>(k_chol_inv_reg<4, 28, true>)};
    for (const void* f : ks) RW_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
    attr = true;
  }
  const size_t sh = chol_reg_lds_bytes(n);
  if (n <= 64)
    k_chol_inv_reg<1, 8, false><<<1, kCholRegThreads, sh, s>>>(G, n, W, info);
  else if (n <= 128)
    k_chol_inv_reg<2, 16, false><<<1, kCholRegThreads, sh, s>>>(G, n, W, info);
  else if (n <= 192)
    k_chol_inv_reg<3, 24, false><<<1, kCholRegThreads, sh, s>>>(G, n, W, info);
  else if (n <= kCholInvMaxN)
    k_chol_inv_reg<4, 25, false><<<1, kCholRegThreads, sh, s>>>(G, n, W, info);
  else
    k_chol_inv_reg<4, 28, true><<<1, kCholRegThreads, sh, s>>>(G, n, W, info);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// Symmetric eigendecomposition by the cyclic Jacobi method with the round-robin ("tournament")
// ordering (Golub & Van Loan, Sec. 8.5): each round rotates n/2 disjoint index pairs at once.
// With J the product of the round's rotations, J^T A J splits into independent 2 x 2 blocks: the
// block of pairs (P1, P2) becomes J1^T A[P1,P2] J2, and the diagonal block of a pair becomes
// diag(a_pp - t a_pq, a_qq + t a_pq).  One thread updates one 2 x 2 block, so a round is one pass
// over the matrix with no strided row/column sweeps.  The matrix lives in LDS (packed upper
// triangle) when it fits, else in global memory (L2-resident).  Right-hand sides are rotated along
// (giving V^T R), and the rotations are logged so that a second kernel can replay them into V with
// rows spread over several workgroups.  Sweeps stop when a sweep performs no rotation.
// ---------------------------------------------------------------------------------------------
constexpr int kJacobiThreads = 1024;
constexpr int kJacobiMaxSweeps = 30;
constexpr int kJacobiBlocksPerThread = 5;   // LDS variant: off-diagonal 2 x 2 blocks held per thread

__device__ __forceinline__ int rr_player(int pos, int round, int n2) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (n2 - 1);
}

struct GlbStore {   // full n2 x n2 column-major copy in global memory
  __device__ static void sync() { __syncthreads(); }
  double* a;
  int n2;
  __device__ __forceinline__ double ld(int i, int j) const { return a[i + j * n2]; }
  __device__ __forceinline__ void st_sym(int i, int j, double v) const {
    a[i + j * n2] = v;
    a[j + i * n2] = v;
  }
};

__host__ __device__ size_t syev_log_count(int n) {
  int n2 = n + (n & 1);
  return (size_t)kJacobiMaxSweeps * (n2 - 1) * (n2 / 2) * 2;
}

// per-matrix work: [glb copy n2*n2][log: (c, s) per round and pair][perm n][sweeps 8][rhs n2*nrhs (global variant)]
static size_t syev_stride(int n, bool vectors, bool glb, int nrhs) {
  int n2 = n + (n & 1);
  size_t s = glb ? (size_t)n2 * n2 : 0;
  if (vectors) s += syev_log_count(n);
  s += n + 8;
  if (glb) s += (size_t)n2 * nrhs;
  return (s + 31) / 32 * 32;
}

// LDS variant: the position-layout matrix, the round's (c, s) pairs and the right-hand sides
__host__ __device__ inline size_t lds_cs_offset(int n) { return (size_t)((JacLayout(n).words() + 1) & ~1); }   // in doubles
static size_t lds_bytes(int n, int nrhs) {
  const JacLayout P(n);
  if ((int64_t)P.nto > (int64_t)kJacobiThreads * kJacobiBlocksPerThread || P.words() >= 32768) return SIZE_MAX;
  return (lds_cs_offset(n) + 2 * (size_t)P.np + (size_t)P.n2 * nrhs) * sizeof(double);
}

size_t syev_work_count(int n, int count, bool vectors, int nrhs) {
  bool glb = lds_bytes(n, nrhs) > kLdsLimit;
  return syev_stride(n, vectors, glb, nrhs) * count;
}

template <class Store>
__device__ void jacobi_body(Store S, int n, int n2, double* rhs, int nrhs, double* log, double* wout, double* permout,
                            double* sweeps_out, double* cs, double* sn, int* pq, double min_rel_tol) {
  const int np = n2 / 2;
  __shared__ int rotated;
  __shared__ double fro_s;
  // Frobenius norm (one wave, fixed order) for the absolute threshold
  if (threadIdx.x < 64) {
    double acc = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = threadIdx.x; i < n; i += 64) {
        double v = S.ld(i, j);
        acc += v * v;
      }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (threadIdx.x == 0) fro_s = sqrt(acc);
  }
  Store::sync();
  // thresholds: rounding noise regenerates off-diagonal entries of size ~eps |A|, so rotations below
  // sqrt(n) eps relative to the diagonal, or eps |A|_F absolute, are skipped; a sweep without
  // rotations ends the iteration
  const double abs_tiny = fro_s * 2.3e-16 + 1e-300;
  const double rel_tol = fmax(2.3e-16 * sqrt((double)n) * 2.0, min_rel_tol);
  const int ta = threadIdx.x & 31, tb = threadIdx.x >> 5;   // 32 x 32 thread grid over pair blocks
  int sweep = 0;
  for (; sweep < kJacobiMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    Store::sync();
    for (int round = 0; round < n2 - 1; ++round) {
      for (int k = threadIdx.x; k < np; k += kJacobiThreads) {
        int p = rr_player(k, round, n2), q = rr_player(n2 - 1 - k, round, n2);
        const bool swapped = p > q;
        if (swapped) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          double apq = S.ld(p, q), app = S.ld(p, p), aqq = S.ld(q, q);
          if (fabs(apq) > abs_tiny && fabs(apq) > rel_tol * sqrt(fabs(app) * fabs(aqq))) {
            double tau = (aqq - app) / (2.0 * apq);
            double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            S.st_sym(p, p, app - t * apq);
            S.st_sym(q, q, aqq + t * apq);
            S.st_sym(p, q, 0.0);
            rotated = 1;
          }
        }
        cs[k] = c;
        sn[k] = s;
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
        if (log) {   // sine of the rotation of (low position, high position)
          double* L = log + ((size_t)(sweep * (n2 - 1) + round) * np + k) * 2;
          L[0] = c;
          L[1] = swapped ? -s : s;
        }
      }
      Store::sync();
      // off-diagonal 2 x 2 blocks of pairs k1 < k2 on a 32 x 32 thread grid (ta = k1 mod 32,
      // tb = k2 mod 32).  Four blocks are loaded before any is stored so that memory latency
      // overlaps; all per-block values stay in registers (constant indices after unrolling).
      // Both stores keep a zero-padded dummy index (odd n) at zero.
      {
        for (int k2 = tb; k2 < np; k2 += 32) {
          const double c2 = cs[k2], s2 = sn[k2];
          const int p2 = pq[2 * k2], q2 = pq[2 * k2 + 1];
          for (int k1b = ta; k1b < k2; k1b += 128) {
            double b0[4], b1[4], b2[4], b3[4], c1[4], s1[4];
            int p1[4], q1[4];
            bool v[4];
  #pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int k1 = k1b + 32 * u;
              const bool in = k1 < k2;
              const int kk = in ? k1 : k2;
              c1[u] = cs[kk];
              s1[u] = sn[kk];
              p1[u] = pq[2 * kk];
              q1[u] = pq[2 * kk + 1];
              v[u] = in && !(s1[u] == 0.0 && s2 == 0.0);
              b0[u] = S.ld(p1[u], p2);
              b1[u] = S.ld(p1[u], q2);
              b2[u] = S.ld(q1[u], p2);
              b3[u] = S.ld(q1[u], q2);
            }
  #pragma unroll
            for (int u = 0; u < 4; ++u) {
              const double r00 = c1[u] * b0[u] - s1[u] * b2[u], r01 = c1[u] * b1[u] - s1[u] * b3[u];  // J1^T B
              const double r10 = s1[u] * b0[u] + c1[u] * b2[u], r11 = s1[u] * b1[u] + c1[u] * b3[u];
              if (v[u]) {
                S.st_sym(p1[u], p2, c2 * r00 - s2 * r01);                                            // (J1^T B) J2
                S.st_sym(p1[u], q2, s2 * r00 + c2 * r01);
                S.st_sym(q1[u], p2, c2 * r10 - s2 * r11);
                S.st_sym(q1[u], q2, s2 * r10 + c2 * r11);
              }
            }
          }
        }
      }
      if (rhs) {
        for (int t = threadIdx.x; t < np * nrhs; t += kJacobiThreads) {
          int k = t % np, r = t / np;
          double s = sn[k];
          if (s == 0.0) continue;
          double c = cs[k];
          int p = pq[2 * k], q = pq[2 * k + 1];
          double vp = rhs[p + r * n2], vq = rhs[q + r * n2];
          rhs[p + r * n2] = c * vp - s * vq;
          rhs[q + r * n2] = s * vp + c * vq;
        }
      }
      Store::sync();
    }
    const int any = rotated;
    Store::sync();
    if (!any) { ++sweep; break; }
  }
  // eigenvalues ascending (stable by index); perm[i] = sorted position of index i
  for (int i = threadIdx.x; i < n; i += kJacobiThreads) {
    double wi = S.ld(i, i);
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      double wj = S.ld(j, j);
      rank += (wj < wi) || (wj == wi && j < i);
    }
    wout[rank] = wi;
    permout[i] = (double)rank;
  }
  if (threadIdx.x == 0) sweeps_out[0] = (double)sweep;
}

// LDS variant (n <= 200): the matrix in the position layout (jacobi_layout.h).  A round is three
// phases separated by workgroup barriers: (1) thread k computes pair k's rotation from its diagonal
// block, (2) every thread rotates its off-diagonal blocks (a fixed set, held in registers) and the
// right-hand sides, (3) every entry is written to its next-round position.  Lanes of a wave touch
// consecutive blocks, so the LDS accesses are free of bank conflicts.  The rotation rule, thresholds
// and log (c and the sine for the (low, high) position order) are those of the global-memory variant; a sweep runs
// only while some off-diagonal entry is above the thresholds, which is the same test as a sweep
// without rotations, evaluated on the matrix at the sweep boundary.
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi_lds(const double* As, int n, double* ws, double* Rs, int nrhs,
                                                                double* work, int64_t stride, int want_log,
                                                                double min_rel_tol) {
  extern __shared__ double smem[];
  const JacLayout P(n);
  const int n2 = P.n2, np = P.np, nto = P.nto;
  const double* A = As + (int64_t)blockIdx.x * n * n;
  double* wk = work + (int64_t)blockIdx.x * stride;
  double* log = want_log ? wk : nullptr;
  double* perm = wk + (want_log ? syev_log_count(n) : 0);
  double* a = smem;
  double* dg = a + 4 * nto;                                            // diagonal blocks: aa, ab, bb
  double2* cs = reinterpret_cast<double2*>(smem + lds_cs_offset(n));  // (c, s) in slot convention
  double* rhs = reinterpret_cast<double*>(cs + np);
  __shared__ int big;
  __shared__ double fro_s;
  for (int t = threadIdx.x; t < P.words(); t += kJacobiThreads) a[t] = 0.0;
  __syncthreads();
  // at a sweep boundary position x holds index x
  for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += kJacobiThreads) {
    const int i = (int)(t % n), j = (int)(t / n);
    if (i <= j) a[P.at(i, j)] = 0.5 * (A[t] + A[j + (int64_t)i * n]);
  }
  double* R = Rs ? Rs + (int64_t)blockIdx.x * n * nrhs : nullptr;
  if (R)
    for (int64_t t = threadIdx.x; t < (int64_t)n2 * nrhs; t += kJacobiThreads) {
      const int i = (int)(t % n2), r = (int)(t / n2);
      rhs[t] = i < n ? R[i + (int64_t)r * n] : 0.0;
    }
  __syncthreads();
  if (threadIdx.x < 64) {   // Frobenius norm, one wave, fixed order
    double acc = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = threadIdx.x; i < n; i += 64) {
        const double v = a[P.at(i, j)];
        acc += v * v;
      }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (threadIdx.x == 0) fro_s = sqrt(acc);
  }
  // this thread's off-diagonal blocks and the flat indices their entries move to after a round
  // (flat indices are below 2^15 at n <= 200, so two share a register)
  int blk[kJacobiBlocksPerThread], kk[kJacobiBlocksPerThread], dst[kJacobiBlocksPerThread][2];
#pragma unroll
  for (int u = 0; u < kJacobiBlocksPerThread; ++u) {
    const int L = threadIdx.x + u * kJacobiThreads;
    blk[u] = -1;
    kk[u] = 0;
    dst[u][0] = dst[u][1] = 0;
    if (L < nto) {
      int k1, k2;
      P.unfold(L, k1, k2);
      blk[u] = P.block(k1, k2);
      kk[u] = k1 | (k2 << 16);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        dst[u][e >> 1] |= P.at(P.next(P.pos(k1, e >> 1)), P.next(P.pos(k2, e & 1))) << (16 * (e & 1));
    }
  }
  int ddst[2] = {0, 0};
  if (threadIdx.x < np) {
    const int k = threadIdx.x;
    ddst[0] = P.at(P.next(P.pos(k, 0)), P.next(P.pos(k, 0))) | (P.at(P.next(P.pos(k, 0)), P.next(P.pos(k, 1))) << 16);
    ddst[1] = P.at(P.next(P.pos(k, 1)), P.next(P.pos(k, 1)));
  }
  __syncthreads();
  // thresholds: rounding noise regenerates off-diagonal entries of size ~eps |A|, so rotations below
  // sqrt(n) eps relative to the diagonal, or eps |A|_F absolute, are skipped
  const double abs_tiny = fro_s * 2.3e-16 + 1e-300;
  const double rel_tol = fmax(2.3e-16 * sqrt((double)n) * 2.0, min_rel_tol);
  auto above = [&](double v, double d1, double d2) {
    return fabs(v) > abs_tiny && fabs(v) > rel_tol * sqrt(fabs(d1) * fabs(d2));
  };
  int sweep = 0;
  for (; sweep < kJacobiMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) big = 0;
    lds_barrier();
    int mine = 0;
#pragma unroll
    for (int u = 0; u < kJacobiBlocksPerThread; ++u)
      if (blk[u] >= 0) {
        const int k1 = kk[u] & 0xffff, k2 = kk[u] >> 16;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          mine |= above(a[e * nto + blk[u]], dg[(e >> 1) * 2 * np + k1], dg[(e & 1) * 2 * np + k2]);
      }
    if (threadIdx.x < np) {
      const int k = threadIdx.x;
      mine |= (n2 - 1 - k < n) && above(dg[np + k], dg[k], dg[2 * np + k]);
    }
    if (mine) big = 1;
    lds_barrier();
    if (!big) break;
    for (int round = 0; round < n2 - 1; ++round) {
      // (1) rotations from the diagonal blocks (index convention p < q for the thresholds and the log)
      double daa = 0.0, dab = 0.0, dbb = 0.0;
      if (threadIdx.x < np) {
        const int k = threadIdx.x;
        const int pa = rr_player(k, round, n2), pb = rr_player(n2 - 1 - k, round, n2);
        daa = dg[k];
        dab = dg[np + k];
        dbb = dg[2 * np + k];
        const bool low = pa < pb;   // the low position holds p
        const double app = low ? daa : dbb, aqq = low ? dbb : daa, apq = dab;
        double c = 1.0, s = 0.0;
        if ((low ? pb : pa) < n && above(apq, app, aqq)) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          const double np_ = app - t * apq, nq_ = aqq + t * apq;
          daa = low ? np_ : nq_;
          dbb = low ? nq_ : np_;
          dab = 0.0;
        }
        const double2 rot = make_double2(c, low ? s : -s);   // with p and q exchanged the sine flips
        cs[k] = rot;
        if (log) *reinterpret_cast<double2*>(log + ((size_t)(sweep * (n2 - 1) + round) * np + k) * 2) = rot;
      }
      lds_barrier();
      // (2) J1^T B J2 for this thread's blocks; right-hand sides.  The empty asm statements mark the
      // array stride and the packed destinations as changing every round, so that the compiler does
      // not keep twenty precomputed addresses live across the loop (which would spill registers).
      int nto_r = nto;
      asm volatile("" : "+s"(nto_r));
      double v[kJacobiBlocksPerThread][4];
#pragma unroll
      for (int u = 0; u < kJacobiBlocksPerThread; ++u)
        if (blk[u] >= 0) {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[u][e] = a[e * nto_r + blk[u]];
          const double2 r1 = cs[kk[u] & 0xffff], r2 = cs[kk[u] >> 16];
          if (!(r1.y == 0.0 && r2.y == 0.0)) {
            const double c1 = r1.x, s1 = r1.y, c2 = r2.x, s2 = r2.y;
            const double r00 = c1 * v[u][0] - s1 * v[u][2], r01 = c1 * v[u][1] - s1 * v[u][3];
            const double r10 = s1 * v[u][0] + c1 * v[u][2], r11 = s1 * v[u][1] + c1 * v[u][3];
            v[u][0] = c2 * r00 - s2 * r01;
            v[u][1] = s2 * r00 + c2 * r01;
            v[u][2] = c2 * r10 - s2 * r11;
            v[u][3] = s2 * r10 + c2 * r11;
          }
        }
      if (R) {
        for (int t = threadIdx.x; t < np * nrhs; t += kJacobiThreads) {
          const int k = t % np, r = t / np;
          const double2 rot = cs[k];
          if (rot.y == 0.0) continue;
          const int x = rr_player(k, round, n2), y = rr_player(n2 - 1 - k, round, n2);
          const double vx = rhs[x + r * n2], vy = rhs[y + r * n2];
          rhs[x + r * n2] = rot.x * vx - rot.y * vy;
          rhs[y + r * n2] = rot.y * vx + rot.x * vy;
        }
      }
      lds_barrier();
      // (3) move every entry to its next-round position
#pragma unroll
      for (int u = 0; u < kJacobiBlocksPerThread; ++u)
        if (blk[u] >= 0) {
          asm volatile("" : "+v"(dst[u][0]), "+v"(dst[u][1]));
#pragma unroll
          for (int e = 0; e < 4; ++e) a[(dst[u][e >> 1] >> (16 * (e & 1))) & 0xffff] = v[u][e];
        }
      if (threadIdx.x < np) {
        a[ddst[0] & 0xffff] = daa;
        a[ddst[0] >> 16] = dab;
        a[ddst[1]] = dbb;
      }
      lds_barrier();
    }
  }
  // eigenvalues ascending (stable by index); perm[i] = sorted position of index i
  double* wout = ws + (int64_t)blockIdx.x * n;
  for (int i = threadIdx.x; i < n; i += kJacobiThreads) {
    const double wi = a[P.at(i, i)];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = a[P.at(j, j)];
      rank += (wj < wi) || (wj == wi && j < i);
    }
    wout[rank] = wi;
    perm[i] = (double)rank;
  }
  if (threadIdx.x == 0) perm[n] = (double)sweep;
  __syncthreads();
  if (R)
    for (int64_t t = threadIdx.x; t < (int64_t)n * nrhs; t += kJacobiThreads) {
      const int i = (int)(t % n), r = (int)(t / n);
      R[(int)perm[i] + (int64_t)r * n] = rhs[i + (int64_t)r * n2];
    }
}

__global__ __launch_bounds__(kJacobiThreads) void k_jacobi_glb(const double* As, int n, double* ws, double* Rs, int nrhs,
                                                                double* work, int64_t stride, int want_log,
                                                                double min_rel_tol) {
  const int n2 = n + (n & 1);
  __shared__ double cs[512], sn[512];
  __shared__ int pq[1024];
  const double* A = As + (int64_t)blockIdx.x * n * n;
  double* wk = work + (int64_t)blockIdx.x * stride;
  double* a = wk;
  double* log = want_log ? wk + (size_t)n2 * n2 : nullptr;
  double* perm = wk + (size_t)n2 * n2 + (want_log ? syev_log_count(n) : 0);
  double* rhs = perm + n + 8;
  GlbStore S{a, n2};
  for (int64_t t = threadIdx.x; t < (int64_t)n2 * n2; t += kJacobiThreads) {
    int i = (int)(t % n2), j = (int)(t / n2);
    a[t] = (i < n && j < n) ? 0.5 * (A[i + (int64_t)j * n] + A[j + (int64_t)i * n]) : 0.0;
  }
  double* R = Rs ? Rs + (int64_t)blockIdx.x * n * nrhs : nullptr;
  if (R)
    for (int64_t t = threadIdx.x; t < (int64_t)n2 * nrhs; t += kJacobiThreads) {
      int i = (int)(t % n2), r = (int)(t / n2);
      rhs[t] = i < n ? R[i + (int64_t)r * n] : 0.0;
    }
  __syncthreads();
  jacobi_body(S, n, n2, R ? rhs : nullptr, nrhs, log, ws + (int64_t)blockIdx.x * n, perm, perm + n, cs, sn, pq,
              min_rel_tol);
  __syncthreads();
  if (R)
    for (int64_t t = threadIdx.x; t < (int64_t)n * nrhs; t += kJacobiThreads) {
      int i = (int)(t % n), r = (int)(t / n);
      R[(int)perm[i] + (int64_t)r * n] = rhs[i + (int64_t)r * n2];
    }
}

// V from the logged rotations: V = J(1) J(2) ... applied to the identity.  Rows of V are independent
// and are replayed in the position layout of jacobi_layout.h: lane l holds, for each of its PPL pairs
// k = l PPL + j, the row's entries at the pair's low and high positions, so a rotation touches only the
// lane's own registers, and the move to the next round's positions shifts low-slot entries down one pair
// and high-slot entries up one pair (one cross-lane shuffle each).  One wave replays R rows; the logged
// (c, s) of upcoming rounds are loaded D rounds ahead.  After whole sweeps position x holds index x, and
// the columns are written in sorted order.
template <int PPL, int R, int D>
__global__ __launch_bounds__(64) void k_jacobi_replay(int n, const double* work, int64_t stride, int64_t log_off,
                                                      double* Vs) {
  const int n2 = n + (n & 1), np = n2 / 2;
  const int b = blockIdx.y;
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * R;
  const double* wk = work + (int64_t)b * stride;
  const double2* log = reinterpret_cast<const double2*>(wk + log_off);
  const double* perm = wk + log_off + syev_log_count(n);
  const int total = (int)perm[n] * (n2 - 1);
  double va[R][PPL], vb[R][PPL];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const int k = lane * PPL + j;
      va[r][j] = (k < np && k == r0 + r) ? 1.0 : 0.0;
      vb[r][j] = (k < np && n2 - 1 - k == r0 + r) ? 1.0 : 0.0;
    }
  auto fetch = [&](int g, double2 (&dst)[PPL]) {
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const int k = lane * PPL + j;
      dst[j] = (g < total && k < np) ? log[(size_t)g * np + k] : make_double2(1.0, 0.0);
    }
  };
  double2 q[D][PPL];
#pragma unroll
  for (int d = 0; d < D; ++d) fetch(d, q[d]);
  for (int g0 = 0; g0 < total; g0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int g = g0 + d;
      if (g >= total) break;   // uniform across the wave
      double2 rot[PPL];
#pragma unroll
      for (int j = 0; j < PPL; ++j) rot[j] = q[d][j];
      fetch(g + D, q[d]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          const double x = va[r][j], y = vb[r][j];
          va[r][j] = rot[j].x * x - rot[j].y * y;
          vb[r][j] = rot[j].y * x + rot[j].x * y;
        }
        if (np > 1) {
          // low slot of pair k <- low slot of pair k+1; high slot of pair k <- high slot of pair k-1;
          // pair 0 keeps its low entry and takes pair 1's; the last pair's low slot takes its high entry
          const double from_next = __shfl_down(va[r][0], 1);
          const double from_prev = __shfl_up(vb[r][PPL - 1], 1);
          double na[PPL], nb[PPL];
#pragma unroll
          for (int j = 0; j < PPL; ++j) {
            const int k = lane * PPL + j;
            const double up = j + 1 < PPL ? va[r][j + 1] : from_next;
            const double dn = j > 0 ? vb[r][j - 1] : from_prev;
            na[j] = k == 0 ? va[r][j] : (k == np - 1 ? vb[r][j] : up);
            nb[j] = k == 0 ? up : dn;
          }
#pragma unroll
          for (int j = 0; j < PPL; ++j) {
            va[r][j] = na[j];
            vb[r][j] = nb[j];
          }
        }
      }
    }
  }
  double* V = Vs + (int64_t)b * n * n;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int row = r0 + r;
    if (row >= n) break;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const int k = lane * PPL + j;
      if (k >= np) continue;
      if (k < n) V[row + (int64_t)((int)perm[k]) * n] = va[r][j];
      const int x = n2 - 1 - k;
      if (x < n) V[row + (int64_t)((int)perm[x]) * n] = vb[r][j];
    }
  }
}

template <int PPL, int R, int D>
static void launch_replay(int n, int count, const double* work, int64_t stride, int64_t log_off, double* V,
                          hipStream_t s) {
  dim3 grid((n + R - 1) / R, count);
  k_jacobi_replay<PPL, R, D><<<grid, 64, 0, s>>>(n, work, stride, log_off, V);
}

int syev_batched(const double* A, double* w, double* V, double* R, int nrhs, int n, int count, double* work,
                 hipStream_t s, double min_rel_tol) {
  if (n <= 0 || count <= 0) return RW_OK;
  RW_CHECK(n <= 1022, RW_EINVAL, "Jacobi eigensolver limited to n <= 1022 (got %d)", n);
  const bool vectors = V != nullptr;
  const int nr = R ? nrhs : 0;
  const bool glb = lds_bytes(n, nr) > kLdsLimit;
  const int64_t stride = (int64_t)syev_stride(n, vectors, glb, nr);
  if (glb) {
    k_jacobi_glb<<<count, kJacobiThreads, 0, s>>>(A, n, w, R, nr, work, stride, vectors ? 1 : 0, min_rel_tol);
  } else {
    size_t sh = lds_bytes(n, R ? nrhs : 0);
    static bool attr_set = false;
    if (!attr_set) {
      RW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_jacobi_lds),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
      attr_set = true;
    }
    k_jacobi_lds<<<count, kJacobiThreads, sh, s>>>(A, n, w, R, R ? nrhs : 0, work, stride, vectors ? 1 : 0,
                                                   min_rel_tol);
  }
  RW_LAUNCH_CHECK();
  if (vectors) {
    const int np = (n + (n & 1)) / 2;
    const int64_t log_off = glb ? (int64_t)(n + (n & 1)) * (n + (n & 1)) : 0;
    // the rotations are loaded 16 (or 8) rounds ahead: a round takes a few hundred cycles, a load from L2
    // or HBM some thousands
    if (np <= 64) launch_replay<1, 2, 16>(n, count, work, stride, log_off, V, s);
    else if (np <= 128) launch_replay<2, 2, 16>(n, count, work, stride, log_off, V, s);
    else if (np <= 256) launch_replay<4, 1, 8>(n, count, work, stride, log_off, V, s);
    else launch_replay<8, 1, 8>(n, count, work, stride, log_off, V, s);
    RW_LAUNCH_CHECK();
  }
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// LU with partial pivoting and solve, one workgroup: A (n x n) and B (n x nrhs) column-major.
// Pivot search by wave 0 (ties -> lowest row).  stat[0] = min |pivot| / max |a_ij|, or 0 when a
// pivot falls below 1e-14 max |a_ij| (the solve is then abandoned).
// ---------------------------------------------------------------------------------------------
__device__ void lu_body(double* A, int n, double* B, int nrhs, double* stat) {
  __shared__ double s_amax, s_minpiv;
  __shared__ int s_prow, s_bad;
  if (threadIdx.x < 64) {
    double m = 0.0;
    for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += 64) m = fmax(m, fabs(A[t]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if (threadIdx.x == 0) { s_amax = m; s_minpiv = INFINITY; s_bad = 0; }
  }
  __syncthreads();
  const double amax = s_amax;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x < 64) {
      double best = -1.0;
      int brow = n;
      for (int i = k + threadIdx.x; i < n; i += 64) {
        double v = fabs(A[i + (int64_t)k * n]);
        if (v > best || (v == best && i < brow)) { best = v; brow = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o);
        int orow = __shfl_xor(brow, o);
        if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; }
      }
      if (threadIdx.x == 0) {
        s_prow = brow;
        if (!(best > 1e-14 * amax)) s_bad = 1;
        s_minpiv = fmin(s_minpiv, best);
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int p = s_prow;
    if (p != k) {
      for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double t = A[k + (int64_t)j * n];
        A[k + (int64_t)j * n] = A[p + (int64_t)j * n];
        A[p + (int64_t)j * n] = t;
      }
      for (int r = threadIdx.x; r < nrhs; r += blockDim.x) {
        double t = B[k + (int64_t)r * n];
        B[k + (int64_t)r * n] = B[p + (int64_t)r * n];
        B[p + (int64_t)r * n] = t;
      }
    }
    __syncthreads();
    const double akk = A[k + (int64_t)k * n];
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i + (int64_t)k * n] /= akk;
    __syncthreads();
    const int m = n - k - 1;
    const int64_t work = (int64_t)m * (m + nrhs);
    for (int64_t t = threadIdx.x; t < work; t += blockDim.x) {
      int i = k + 1 + (int)(t % m);
      int j = (int)(t / m);
      double l = A[i + (int64_t)k * n];
      if (j < m) {
        int jj = k + 1 + j;
        A[i + (int64_t)jj * n] -= l * A[k + (int64_t)jj * n];
      } else {
        int r = j - m;
        B[i + (int64_t)r * n] -= l * B[k + (int64_t)r * n];
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (threadIdx.x == 0) stat[0] = 0.0;
    return;
  }
  // back substitution U x = b'
  for (int k = n - 1; k >= 0; --k) {
    const double ukk = A[k + (int64_t)k * n];
    for (int r = threadIdx.x; r < nrhs; r += blockDim.x) B[k + (int64_t)r * n] /= ukk;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < (int64_t)k * nrhs; t += blockDim.x) {
      int i = (int)(t % k), r = (int)(t / k);
      B[i + (int64_t)r * n] -= A[i + (int64_t)k * n] * B[k + (int64_t)r * n];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) stat[0] = s_minpiv / amax;
}

__global__ __launch_bounds__(1024) void k_lu_solve(double* A, int n, double* B, int nrhs, double* stat) {
  lu_body(A, n, B, nrhs, stat);
}

// The same elimination with A and B in LDS (rows padded to an odd stride, so that a row read across
// lanes is free of bank conflicts).  Rows are not exchanged: step k eliminates column k from every row not
// yet chosen as a pivot row (a flag per row) using the chosen row p_k; the pivot search of column k+1 runs in
// one wave during step k, so a column costs one barrier.  Back substitution runs over the pivot order.  Ties
// in the pivot search go to the lowest row index, and the solution is written to B in natural order.
constexpr int kLuLdsMaxRows = 192;   // rows per lane in the elimination grid: 3 x 64
constexpr int kLuWaveRhs = 8;        // back substitution in one wave up to this many right-hand sides

__device__ void lu_lds_body(const double* Ag, int n, double* Bg, int nrhs, double* stat) {
  extern __shared__ double sm[];
  const int ld = n | 1;
  double* A = sm;                       // ld x n
  double* B = A + (size_t)ld * n;       // ld x nrhs
  int* prow = reinterpret_cast<int*>(B + (size_t)ld * nrhs);   // n: pivot row of step k
  int* done = prow + n;                  // n: row already used as a pivot row
  __shared__ double s_amax, s_minpiv;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int t = tid; t < n * n; t += blockDim.x) A[(t % n) + (t / n) * ld] = Ag[t];
  for (int t = tid; t < n * nrhs; t += blockDim.x) B[(t % n) + (t / n) * ld] = Bg[t];
  for (int t = tid; t < n; t += blockDim.x) done[t] = 0;
  __syncthreads();
  if (tid < 64) {
    double m = 0.0;
    for (int t = tid; t < n * n; t += 64) m = fmax(m, fabs(A[(t % n) + (t / n) * ld]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if (tid == 0) { s_amax = m; s_minpiv = INFINITY; s_bad = 0; }
  }
  __syncthreads();
  const double amax = s_amax;
  // pivot of column k (one wave): argmax of |A(i, k)| over rows not yet chosen, ties to the lowest row index;
  // prow[k], the smallest pivot so far, s_bad when no usable pivot is left
  auto pivot = [&](int k) {
    double best = -1.0;
    int brow = n;
    for (int i = lane; i < n; i += 64) {
      if (done[i]) continue;
      const double v = fabs(A[i + k * ld]);
      if (v > best) { best = v; brow = i; }   // rows visited in increasing order: first maximum kept
    }
    const double m = wave_max64(best);
    const unsigned long long tie = __ballot(best == m);
    int row;
    if (__popcll(tie) == 1) {
      row = __shfl(brow, __ffsll((long long)tie) - 1);
    } else {
      int r = best == m ? brow : n;
      for (int o = 32; o > 0; o >>= 1) r = min(r, __shfl_xor(r, o));
      row = r;
    }
    if (lane == 0) {
      const bool ok = row < n && m > 1e-14 * amax;   // no candidate (NaN column) or a tiny pivot
      prow[k] = ok ? row : 0;
      if (!ok) s_bad = 1;
      s_minpiv = fmin(s_minpiv, m);
    }
  };
  if (wave == 0) pivot(0);
  __syncthreads();
  // step k eliminates column k with pivot row p = prow[k]: x(i) -= (A(i,k) / A(p,k)) x(p) on the rows not yet
  // chosen.  Wave 0 updates column k+1 first and finds its pivot while the other waves update columns k+2..
  // and B, so a step costs one barrier.
  for (int k = 0; k < n; ++k) {
    if (s_bad) break;   // uniform
    const int p = prow[k];
    const double inv = 1.0 / A[p + k * ld];
    // rows of the lanes (up to three each); row p is not marked done yet (wave 0 marks it below, and the test
    // i != p excludes it either way)
    double l[3];
    bool act[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int i = lane + 64 * q;
      act[q] = i < n && i != p && !done[i];
      l[q] = act[q] ? A[i + k * ld] * inv : 0.0;
    }
    if (wave == 0) {
      if (lane == 0) done[p] = 1;
      if (k + 1 < n) {
        double* col = A + (k + 1) * ld;
        const double xp = col[p];
#pragma unroll
        for (int q = 0; q < 3; ++q)
          if (act[q]) col[lane + 64 * q] -= l[q] * xp;
        pivot(k + 1);
      }
    } else {
      const int na = n - k - 2 > 0 ? n - k - 2 : 0;   // columns k+2.. of A, then all of B
      const int cols = na + nrhs;
      for (int c = wave - 1; c < cols; c += 15) {
        double* col = c < na ? A + (k + 2 + c) * ld : B + (c - na) * ld;
        const double xp = col[p];
#pragma unroll
        for (int q = 0; q < 3; ++q)
          if (act[q]) col[lane + 64 * q] -= l[q] * xp;
      }
    }
    lds_barrier();
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) stat[0] = 0.0;
    return;
  }
  // back substitution over the pivot order: x_k = b(p_k) / A(p_k, k); b(p_i) -= A(p_i, k) x_k for i < k
  if (nrhs <= kLuWaveRhs) {
    // one wave, lanes over the pivot order positions i (up to three each), the right-hand sides of a lane's
    // rows held in registers: b(p_k) is read from the lane holding position k, so a step's chain is a lane
    // read, a product and the lanes' updates, with no LDS round trip and no barriers
    if (wave == 0) {
      int pr[3];
      double bv[3][kLuWaveRhs];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const bool in = lane + 64 * q < n;
        pr[q] = in ? prow[lane + 64 * q] : 0;
#pragma unroll
        for (int r = 0; r < kLuWaveRhs; ++r) bv[q][r] = (in && r < nrhs) ? B[pr[q] + r * ld] : 0.0;
      }
      for (int k = n - 1; k >= 0; --k) {
        const int p = prow[k], kq = k >> 6, kl = k & 63;   // position k: lane kl, slot kq
        const double rukk = 1.0 / A[p + k * ld];
        double a[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) a[q] = lane + 64 * q < k ? A[pr[q] + k * ld] : 0.0;
#pragma unroll
        for (int r = 0; r < kLuWaveRhs; ++r) {
          if (r >= nrhs) break;   // uniform
          // b(p_k) is final: every later step has been applied
          const double bk = lane_read(kq == 0 ? bv[0][r] : (kq == 1 ? bv[1][r] : bv[2][r]), kl);
          const double xk = bk * rukk;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            if (lane + 64 * q < k) bv[q][r] -= a[q] * xk;
            if (q == kq && lane == kl) bv[q][r] = xk;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (lane + 64 * q >= n) continue;
#pragma unroll
        for (int r = 0; r < kLuWaveRhs; ++r)
          if (r < nrhs) B[pr[q] + r * ld] = bv[q][r];
      }
    }
    __syncthreads();
  } else {
    for (int k = n - 1; k >= 0; --k) {
      const int p = prow[k];
      const double ukk = A[p + k * ld];
      for (int r = tid; r < nrhs; r += blockDim.x) B[p + r * ld] /= ukk;
      lds_barrier();
      for (int t = tid; t < k * nrhs; t += blockDim.x) {
        const int i = t % k, r = t / k;
        const int pi = prow[i];
        B[pi + r * ld] -= A[pi + k * ld] * B[p + r * ld];
      }
      lds_barrier();
    }
  }
  for (int t = tid; t < n * nrhs; t += blockDim.x) {
    const int k = t % n, r = t / n;
    Bg[k + (int64_t)r * n] = B[prow[k] + r * ld];
  }
  if (tid == 0) stat[0] = s_minpiv / amax;
}

// ---------------------------------------------------------------------------------------------
// Register-resident LU for n <= 32 R (R <= kLuRegMaxR), used where the LDS elimination below does not fit
// (its trailing block no longer fits in LDS, n > 141 or so): the 1024 threads form a 32 x 32 grid and thread
// (ti, tj) holds the elements (ti + 32 r, tj + 32 c) of A in registers; only B (n x nrhs), the step's
// multipliers and pivot row, and the pivots live in LDS.  The elimination is that of lu_lds_body (same pivot
// choice: largest magnitude over the rows not yet chosen, ties to the lowest row; the same products, so the
// same bits); a step costs two barriers and a handful of LDS reads per thread instead of a sweep of the
// trailing block through LDS.  The pivot of column k+1 is found by the 32 threads holding that column, in
// one half-wave, right after their update.  Back substitution by the 32 threads holding column k.
// Measured per step (one workgroup, n = 75 / 150): 2.4 / 3.2 us against 1.7 us for the LDS elimination and
// 6.3 us for the global one; a workgroup barrier alone costs about 0.15 us and a dependent LDS read about
// 0.07 us, so the step is latency-bound either way.  Beyond R = 6 the register tile spills.
// ---------------------------------------------------------------------------------------------
constexpr int kLuRegMaxR = 6;   // n <= 192

__host__ __device__ inline size_t lu_reg_bytes(int n, int nrhs) {
  return ((size_t)(n | 1) * nrhs + 3 * (size_t)n + 18) * sizeof(double) + (size_t)n * sizeof(int);
}
__host__ __device__ inline bool lu_reg_fits(int n, int nrhs) {
  return n <= 32 * kLuRegMaxR && lu_reg_bytes(n, nrhs) <= kLdsLimit;
}

template <int R>
__device__ void lu_reg_body(const double* Ag, int n, double* Bg, int nrhs, double* stat) {
  extern __shared__ double sm[];
  const int ld = n | 1;
  double* B = sm;                              // ld x nrhs
  double* colbuf = B + (size_t)ld * nrhs;      // n: multipliers of the step (0 on rows not eliminated)
  double* rowbuf = colbuf + n;                 // n: the pivot row
  double* diag = rowbuf + n;                   // n: u(p_k, k)
  double* s_wmax = diag + n;                   // 16: per-wave maxima
  double& s_minpiv = s_wmax[16];
  int& s_bad = *reinterpret_cast<int*>(s_wmax + 17);
  int* prow = reinterpret_cast<int*>(s_wmax + 18);   // n: pivot row of step k
  // (the scalars live in the dynamic allocation: the batched kernel's static LDS stays within what its
  // dynamic size leaves)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ti = lane & 31, tj = 2 * wave + (lane >> 5);
  double a[R][R];
  int rpos[R];   // the step at which row ti + 32 r became the pivot row, n before
  // a[r][c] with a run-time c (or r), by unrolled selects: a run-time index into the register array would
  // move it to scratch memory
  auto col_of = [&](int r, int cs) {
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < R; ++c) v = c == cs ? a[r][c] : v;
    return v;
  };
  double amax = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    rpos[r] = n;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int i = ti + 32 * r, j = tj + 32 * c;
      a[r][c] = (i < n && j < n) ? Ag[i + (int64_t)j * n] : 0.0;
      amax = fmax(amax, fabs(a[r][c]));
    }
  }
  for (int t = tid; t < n * nrhs; t += blockDim.x) B[(t % n) + (t / n) * ld] = Bg[t];
  amax = wave_max64(amax);
  if (lane == 0) s_wmax[wave] = amax;
  if (tid == 0) {
    s_minpiv = INFINITY;
    s_bad = 0;
  }
  __syncthreads();
  amax = s_wmax[0];
  for (int w = 1; w < 16; ++w) amax = fmax(amax, s_wmax[w]);
  // pivot of column k by the half-wave holding it (tj == k mod 32): largest |a| over the rows not yet chosen,
  // ties to the lowest row
  auto pivot = [&](int k) {
    const int cs = k >> 5;
    double best = -1.0, val = 0.0;
    int brow = n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = ti + 32 * r;
      const double v = col_of(r, cs);
      if (i < n && rpos[r] == n && fabs(v) > best) {   // rows in increasing order: first maximum kept
        best = fabs(v);
        val = v;
        brow = i;
      }
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o), ov = __shfl_xor(val, o);
      const int orow = __shfl_xor(brow, o);
      if (ob > best || (ob == best && orow < brow)) {
        best = ob;
        val = ov;
        brow = orow;
      }
    }
    if (ti == 0) {
      const bool ok = brow < n && best > 1e-14 * amax;
      prow[k] = ok ? brow : 0;
      diag[k] = ok ? val : 1.0;
      if (!ok) s_bad = 1;
      s_minpiv = fmin(s_minpiv, best);
    }
  };
  if (tj == 0) pivot(0);
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (s_bad) break;   // uniform
    const int p = prow[k];
    const double inv = 1.0 / diag[k];
    // the multipliers of column k and the pivot row
    if (tj == (k & 31)) {
      const int cs = k >> 5;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = ti + 32 * r;
        if (i < n) colbuf[i] = (rpos[r] == n && i != p) ? col_of(r, cs) * inv : 0.0;
      }
    }
    if (ti == (p & 31)) {
      const int rs = p >> 5;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const int j = tj + 32 * c;
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) v = r == rs ? a[r][c] : v;
        if (j > k && j < n) rowbuf[j] = v;
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r == rs) rpos[r] = k;
    }
    lds_barrier();
    // the update of the rows not yet chosen, then B, then the next pivot
    double rb[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int j = tj + 32 * c;
      rb[c] = (j > k && j < n) ? rowbuf[j] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = ti + 32 * r;
      if (i < n && rpos[r] == n) {
        const double l = colbuf[i];
#pragma unroll
        for (int c = 0; c < R; ++c) {
          const int j = tj + 32 * c;
          if (j > k && j < n) a[r][c] -= l * rb[c];
        }
      }
    }
    for (int t = tid; t < n * nrhs; t += blockDim.x) {
      const int i = t % n, q = t / n;
      B[i + q * ld] -= colbuf[i] * B[p + q * ld];
    }
    if (k + 1 < n && tj == ((k + 1) & 31)) pivot(k + 1);
    lds_barrier();
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) stat[0] = 0.0;
    return;
  }
  // back substitution over the pivot order: x_k = b(p_k) / u(p_k, k); b(p_i) -= u(p_i, k) x_k for i < k
  for (int k = n - 1; k >= 0; --k) {
    if (tj == (k & 31)) {
      const int p = prow[k], cs = k >> 5;
      const double rukk = 1.0 / diag[k];
      for (int q = 0; q < nrhs; ++q) {
        const double xk = B[p + q * ld] * rukk;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = ti + 32 * r;
          if (i < n && rpos[r] < k) B[i + q * ld] -= col_of(r, cs) * xk;
        }
        if (ti == 0) B[p + q * ld] = xk;
      }
    }
    lds_barrier();
  }
  for (int t = tid; t < n * nrhs; t += blockDim.x) {
    const int k = t % n, q = t / n;
    Bg[k + (int64_t)q * n] = B[prow[k] + q * ld];
  }
  if (tid == 0) stat[0] = s_minpiv / amax;
}

__device__ void lu_reg_dispatch(const double* Ag, int n, double* Bg, int nrhs, double* stat) {
  switch ((n + 31) >> 5) {
    case 1: lu_reg_body<1>(Ag, n, Bg, nrhs, stat); break;
    case 2: lu_reg_body<2>(Ag, n, Bg, nrhs, stat); break;
    case 3: lu_reg_body<3>(Ag, n, Bg, nrhs, stat); break;
    case 4: lu_reg_body<4>(Ag, n, Bg, nrhs, stat); break;
    case 5: lu_reg_body<5>(Ag, n, Bg, nrhs, stat); break;
    default: lu_reg_body<6>(Ag, n, Bg, nrhs, stat); break;
  }
}

template <int R>
__global__ __launch_bounds__(1024) void k_lu_reg(const double* Ag, int n, double* Bg, int nrhs, double* stat) {
  lu_reg_body<R>(Ag, n, Bg, nrhs, stat);
}

// ---------------------------------------------------------------------------------------------
// Register-column LU for 192 < n <= 208, beyond the register tile: column c belongs to wave c % 16, which keeps
// rows 0..127 of it in registers (lane l: rows l and l + 64); rows 128.. of every column live in LDS (lane l:
// rows 128 + l and 192 + l).  The elimination is that of lu_lds_body (no row exchanges; pivot: largest magnitude
// over the rows not yet chosen, ties to the lowest row; the same products).  In step k the owner of column k+1
// updates that column first, copies its register rows to an LDS vector (two, alternating by step) and finds
// its pivot, while the other waves update the columns they own with the multipliers of column k from the
// previous vector and the pivot row's entries read across lanes; one barrier per step.  Back substitution by
// the owner of each column in turn, over the pivot order.
// ---------------------------------------------------------------------------------------------
constexpr int kLuColRegRows = 128;   // rows held in registers (two per lane)
constexpr int kLuColMaxN = 208;      // 13 columns per wave (more spill at 1024 threads)
constexpr int kLuColMinN = 193;      // below, the register tile serves

__host__ __device__ inline size_t lu_col_bytes(int n, int nrhs) {
  const size_t ldl = (size_t)((n - kLuColRegRows) | 1);
  return (ldl * n + (size_t)(n | 1) * nrhs + 2 * kLuColRegRows + 18) * sizeof(double) +
         (3 * (size_t)n + 1) * sizeof(int);
}
__host__ __device__ inline bool lu_col_fits(int n, int nrhs) {
  return n >= kLuColMinN && n <= kLuColMaxN && lu_col_bytes(n, nrhs) <= kLdsLimit;
}

template <int NC>
__device__ void lu_col_body(const double* Ag, int n, double* Bg, int nrhs, double* stat) {
  constexpr int RR = kLuColRegRows;
  extern __shared__ double sm[];
  const int nl = n - RR, ldl = nl | 1, ldb = n | 1;
  double* AL = sm;                              // ldl x n: rows RR.. of every column
  double* B = AL + (size_t)ldl * n;             // ldb x nrhs
  double* nx = B + (size_t)ldb * nrhs;          // 2 x RR: register rows of the step's pivot column
  double* sc = nx + 2 * RR;                     // [0] max |A|, [1] smallest pivot, [2..17] wave maxima
  int* prow = reinterpret_cast<int*>(sc + 18);  // n: pivot row of step k
  int* done = prow + n;                         // n: row already a pivot row
  int* pos = done + n;                          // n: position of a row in the pivot order
  int* bad = pos + n;                           // 1
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double a[NC][2];   // a[j][q] = A(lane + 64 q, wave + 16 j)
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int c = wave + 16 * j;
#pragma unroll
    for (int q = 0; q < 2; ++q) a[j][q] = c < n ? Ag[(lane + 64 * q) + (int64_t)c * n] : 0.0;
  }
  double m = 0.0;
#pragma unroll
  for (int j = 0; j < NC; ++j) m = fmax(m, fmax(fabs(a[j][0]), fabs(a[j][1])));
  for (int t = tid; t < nl * n; t += blockDim.x) {
    const double x = Ag[RR + (t % nl) + (int64_t)(t / nl) * n];
    AL[(t % nl) + (t / nl) * ldl] = x;
    m = fmax(m, fabs(x));
  }
  for (int t = tid; t < n * nrhs; t += blockDim.x) B[(t % n) + (t / n) * ldb] = Bg[t];
  for (int t = tid; t < n; t += blockDim.x) done[t] = 0;
  m = wave_max64(m);
  if (lane == 0) sc[2 + wave] = m;
  __syncthreads();
  if (tid == 0) {
    double mm = 0.0;
    for (int w = 0; w < 16; ++w) mm = fmax(mm, sc[2 + w]);
    sc[0] = mm;
    sc[1] = INFINITY;
    *bad = 0;
  }
  __syncthreads();
  const double amax = sc[0];
  // this lane's LDS rows: RR + lane + 64 s, s < 2, present when below n
  const bool lr0 = lane < nl, lr1 = lane + 64 < nl;
  // pivot of column c (held in col by the calling wave, after its update): its register rows to nx[c & 1], then
  // the largest magnitude over the rows not yet chosen (a lane's rows in increasing order: first maximum kept;
  // ties across lanes to the lowest row)
  auto pivot = [&](int c, const double (&col)[2]) __attribute__((always_inline)) {
    double best = -1.0;
    int brow = n;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = lane + 64 * q;
      nx[(c & 1) * RR + i] = col[q];
      if (!done[i]) {
        const double v = fabs(col[q]);
        if (v > best) { best = v; brow = i; }
      }
    }
    if (lr0 && !done[RR + lane]) {
      const double v = fabs(AL[lane + c * ldl]);
      if (v > best) { best = v; brow = RR + lane; }
    }
    if (lr1 && !done[RR + 64 + lane]) {
      const double v = fabs(AL[lane + 64 + c * ldl]);
      if (v > best) { best = v; brow = RR + 64 + lane; }
    }
    const double mx = wave_max64(best);
    const unsigned long long tie = __ballot(best == mx);
    int row;
    if (__popcll(tie) == 1) {
      row = __shfl(brow, __ffsll((long long)tie) - 1);
    } else {
      int r = best == mx ? brow : n;
      for (int o = 32; o > 0; o >>= 1) r = min(r, __shfl_xor(r, o));
      row = r;
    }
    if (lane == 0) {
      const bool ok = row < n && mx > 1e-14 * amax;
      prow[c] = ok ? row : 0;
      if (!ok) *bad = 1;
      sc[1] = fmin(sc[1], mx);
    }
  };
  if (wave == 0) pivot(0, a[0]);
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (*bad) break;   // uniform
    const int p = prow[k];
    const double* ck = nx + (k & 1) * RR;
    const double inv = 1.0 / (p < RR ? ck[p] : AL[(p - RR) + k * ldl]);
    // multipliers of this lane's rows: registers (lane, lane + 64), LDS (RR + lane, RR + 64 + lane)
    const bool act0 = lane != p && !done[lane], act1 = lane + 64 != p && !done[lane + 64];
    const bool act2 = lr0 && RR + lane != p && !done[RR + lane];
    const bool act3 = lr1 && RR + 64 + lane != p && !done[RR + 64 + lane];
    const double l0 = act0 ? ck[lane] * inv : 0.0, l1 = act1 ? ck[lane + 64] * inv : 0.0;
    const double l2 = act2 ? AL[lane + k * ldl] * inv : 0.0, l3 = act3 ? AL[lane + 64 + k * ldl] * inv : 0.0;
    const bool pr = p < RR;
    const int pl = p & 63;
    auto update = [&](double (&col)[2], int c) __attribute__((always_inline)) {
      const double xp = pr ? __shfl(p < 64 ? col[0] : col[1], pl) : AL[(p - RR) + c * ldl];
      if (act0) col[0] -= l0 * xp;
      if (act1) col[1] -= l1 * xp;
      if (act2) AL[lane + c * ldl] -= l2 * xp;
      if (act3) AL[lane + 64 + c * ldl] -= l3 * xp;
    };
    const int k1 = k + 1;
    if (k1 < n && wave == (k1 & 15)) {   // the next pivot column first, then its pivot
      if (lane == 0) done[p] = 1;
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (j == (k1 >> 4)) {
          update(a[j], k1);
          pivot(k1, a[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c = wave + 16 * j;
      if (c > k1 && c < n) update(a[j], c);
    }
    for (int r = wave; r < nrhs; r += 16) {
      double* col = B + r * ldb;
      const double xp = col[p];
      if (act0) col[lane] -= l0 * xp;
      if (act1) col[lane + 64] -= l1 * xp;
      if (act2) col[RR + lane] -= l2 * xp;
      if (act3) col[RR + 64 + lane] -= l3 * xp;
    }
    __syncthreads();
  }
  if (*bad) {
    if (tid == 0) stat[0] = 0.0;
    return;
  }
  for (int t = tid; t < n; t += blockDim.x) pos[prow[t]] = t;
  __syncthreads();
  // back substitution over the pivot order: x_k = b(p_k) / A(p_k, k); b(p_i) -= A(p_i, k) x_k for i < k, by the
  // owner of column k
  for (int k = n - 1; k >= 0; --k) {
    if (wave == (k & 15)) {
      const int p = prow[k], pl = p & 63;
      const bool up0 = pos[lane] < k, up1 = pos[lane + 64] < k;
      const bool up2 = lr0 && pos[RR + lane] < k, up3 = lr1 && pos[RR + 64 + lane] < k;
      const double a2 = up2 ? AL[lane + k * ldl] : 0.0, a3 = up3 ? AL[lane + 64 + k * ldl] : 0.0;
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (j == (k >> 4)) {
          const double u = p < RR ? __shfl(p < 64 ? a[j][0] : a[j][1], pl) : AL[(p - RR) + k * ldl];
          const double ru = 1.0 / u;
          for (int r = 0; r < nrhs; ++r) {
            double* col = B + r * ldb;
            const double xk = col[p] * ru;
            if (up0) col[lane] -= a[j][0] * xk;
            if (up1) col[lane + 64] -= a[j][1] * xk;
            if (up2) col[RR + lane] -= a2 * xk;
            if (up3) col[RR + 64 + lane] -= a3 * xk;
            if (lane == 0) col[p] = xk;
          }
        }
    }
    __syncthreads();
  }
  for (int t = tid; t < n * nrhs; t += blockDim.x) {
    const int k = t % n, r = t / n;
    Bg[k + (int64_t)r * n] = B[prow[k] + r * ldb];
  }
  if (tid == 0) stat[0] = sc[1] / amax;
}

__device__ void lu_col_dispatch(const double* Ag, int n, double* Bg, int nrhs, double* stat) {
  lu_col_body<(kLuColMaxN + 15) / 16>(Ag, n, Bg, nrhs, stat);
}

__global__ __launch_bounds__(1024) void k_lu_col(const double* Ag, int n, double* Bg, int nrhs, double* stat) {
  lu_col_dispatch(Ag, n, Bg, nrhs, stat);
}

__host__ __device__ inline size_t lu_lds_bytes(int n, int nrhs) {
  const size_t ld = (size_t)(n | 1);
  return (ld * (n + nrhs)) * sizeof(double) + 2 * (size_t)n * sizeof(int);
}
// the LDS elimination serves a system when it fits; the single and the batched solves decide alike, so a
// batched system is solved by the same code as the same system alone
__host__ __device__ inline bool lu_lds_fits(int n, int nrhs) {
  return n <= kLuLdsMaxRows && lu_lds_bytes(n, nrhs) <= kLdsLimit;
}

__global__ __launch_bounds__(1024) void k_lu_solve_lds(const double* Ag, int n, double* Bg, int nrhs, double* stat) {
  lu_lds_body(Ag, n, Bg, nrhs, stat);
}

// one workgroup per job; jobs (and their sizes) are read from device memory, so a captured launch
// stays valid when the jobs are rewritten between replays
__global__ __launch_bounds__(1024) void k_lu_solve_batched(const LuJob* jobs, int count) {
  const LuJob j = jobs[blockIdx.x];
  if (j.n <= 0) return;
  if (lu_lds_fits(j.n, j.nrhs)) lu_lds_body(j.A, j.n, j.B, j.nrhs, j.stat);
  else if (lu_reg_fits(j.n, j.nrhs)) lu_reg_dispatch(j.A, j.n, j.B, j.nrhs, j.stat);
  else if (lu_col_fits(j.n, j.nrhs)) lu_col_dispatch(j.A, j.n, j.B, j.nrhs, j.stat);
  else lu_body(j.A, j.n, j.B, j.nrhs, j.stat);
}

static int lu_attrs() {
  static bool attr = false;
  if (!attr) {
    RW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lu_solve_lds),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
    RW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lu_solve_batched),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
    const void* regs[] = {reinterpret_cast<const void*>(k_lu_reg<1>), reinterpret_cast<const void*>(k_lu_reg<2>),
                          reinterpret_cast<const void*>(k_lu_reg<3>), reinterpret_cast<const void*>(k_lu_reg<4>),
                          reinterpret_cast<const void*>(k_lu_reg<5>), reinterpret_cast<const void*>(k_lu_reg<6>)};
    for (const void* f : regs)
      RW_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
    RW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lu_col), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kLdsLimit));
    attr = true;
  }
  return RW_OK;
}

int lu_solve_batched(const LuJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return RW_OK;
  RW_TRY(lu_attrs());
  k_lu_solve_batched<<<count, 1024, kLdsLimit, s>>>(jobs, count);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

template <int R>
static void launch_lu_reg(double* A, int n, double* B, int nrhs, double* stat, hipStream_t s) {
  k_lu_reg<R><<<1, 1024, lu_reg_bytes(n, nrhs), s>>>(A, n, B, nrhs, stat);
}

int lu_solve(double* A, int n, double* B, int nrhs, double* stat, hipStream_t s) {
  if (n <= 0) return RW_OK;
  if (!lu_lds_fits(n, nrhs) && lu_reg_fits(n, nrhs)) {
    RW_TRY(lu_attrs());
    switch ((n + 31) >> 5) {
      case 1: launch_lu_reg<1>(A, n, B, nrhs, stat, s); break;
      case 2: launch_lu_reg<2>(A, n, B, nrhs, stat, s); break;
      case 3: launch_lu_reg<3>(A, n, B, nrhs, stat, s); break;
      case 4: launch_lu_reg<4>(A, n, B, nrhs, stat, s); break;
      case 5: launch_lu_reg<5>(A, n, B, nrhs, stat, s); break;
      default: launch_lu_reg<6>(A, n, B, nrhs, stat, s); break;
    }
  } else if (lu_lds_fits(n, nrhs)) {
    RW_TRY(lu_attrs());
    k_lu_solve_lds<<<1, 1024, lu_lds_bytes(n, nrhs), s>>>(A, n, B, nrhs, stat);
  } else if (lu_col_fits(n, nrhs)) {
    RW_TRY(lu_attrs());
    k_lu_col<<<1, 1024, lu_col_bytes(n, nrhs), s>>>(A, n, B, nrhs, stat);
  } else {
    k_lu_solve<<<1, 1024, 0, s>>>(A, n, B, nrhs, stat);
  }
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_dense_syev_workspace_bytes(int n, int count, size_t* bytes) {
  RW_CHECK(bytes != nullptr && n >= 1 && n <= 1022 && count >= 1, RW_EINVAL, "bad sizes");
  *bytes = syev_work_count(n, count, true, 0) * sizeof(double);
  return RW_OK;
}

int rw_dense_syev(const double* A, double* w, double* V, int n, int count, void* work, size_t work_bytes,
                  hipStream_t stream) {
  RW_CHECK(A != nullptr && w != nullptr && work != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(n >= 1 && n <= 1022 && count >= 1, RW_EINVAL, "bad sizes");
  size_t need = syev_work_count(n, count, V != nullptr, 0) * sizeof(double);
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "syev workspace too small: %zu < %zu", work_bytes, need);
  return syev_batched(A, w, V, nullptr, 0, n, count, static_cast<double*>(work), stream);
}

int rw_dense_lu_solve(double* A, int n, double* B, int nrhs, double* stat, hipStream_t stream) {
  RW_CHECK(A != nullptr && B != nullptr && stat != nullptr && n >= 1 && nrhs >= 0, RW_EINVAL, "bad argument");
  return lu_solve(A, n, B, nrhs, stat, stream);
}

}  // extern "C"
