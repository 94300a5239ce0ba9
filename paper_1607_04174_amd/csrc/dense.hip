// Small dense FP64 kernels: Cholesky, triangular inverse, symmetric eigendecomposition (cyclic
// Jacobi) and LU with partial pivoting.  One workgroup owns one matrix held in global memory (it
// stays L2-resident at these sizes); batched launches give each matrix its own workgroup.
#include <cmath>

#include "rw_internal.h"

namespace rw {

// ---------------------------------------------------------------------------------------------
// Cholesky A = L L^T (lower, in place; the strict upper triangle is left untouched)
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol(double* As, int n, int* info) {
  double* A = As + (int64_t)blockIdx.x * n * n;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      double akk = A[k + (int64_t)k * n];
      if (!(akk > 0.0) || !isfinite(akk)) bad = k + 1;
      else A[k + (int64_t)k * n] = sqrt(akk);
    }
    __syncthreads();
    if (bad) break;
    const double piv = A[k + (int64_t)k * n];
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i + (int64_t)k * n] /= piv;
    __syncthreads();
    const int m = n - k - 1;
    for (int64_t t = threadIdx.x; t < (int64_t)m * m; t += blockDim.x) {
      int i = k + 1 + (int)(t % m), j = k + 1 + (int)(t / m);
      if (i >= j) A[i + (int64_t)j * n] -= A[i + (int64_t)k * n] * A[j + (int64_t)k * n];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) info[blockIdx.x] = bad;
}

int chol_batched(double* A, int n, int count, int* info, hipStream_t s) {
  if (n <= 0 || count <= 0) return RW_OK;
  k_chol<<<count, 256, 0, s>>>(A, n, info);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// Rinv = (L^T)^{-1}: thread j back-substitutes column j of the upper-triangular inverse.
__global__ void k_upper_inverse(const double* L, double* Rinv, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double* x = Rinv + (int64_t)j * n;
  for (int i = n - 1; i > j; --i) x[i] = 0.0;
  // R(i,k) = L(k,i) = L[k + i*n]
  x[j] = 1.0 / L[j + (int64_t)j * n];
  for (int i = j - 1; i >= 0; --i) {
    double acc = 0.0;
    for (int k = i + 1; k <= j; ++k) acc += L[k + (int64_t)i * n] * x[k];
    x[i] = -acc / L[i + (int64_t)i * n];
  }
}

int chol_upper_inverse(const double* L, double* Rinv, int n, hipStream_t s) {
  if (n <= 0) return RW_OK;
  k_upper_inverse<<<nblocks(n, 64), 64, 0, s>>>(L, Rinv, n);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// Symmetric eigendecomposition by the cyclic Jacobi method with the round-robin ("tournament")
// ordering: each round rotates n/2 disjoint index pairs at once (Golub & Van Loan, Sec. 8.5), all
// rows first, then all columns and the eigenvector accumulator.  Sweeps stop when a sweep performs
// no rotation.  Eigenvalues are returned ascending with their vectors.
// ---------------------------------------------------------------------------------------------
constexpr int kJacobiThreads = 1024;
constexpr int kJacobiMaxSweeps = 40;

__device__ __forceinline__ int rr_player(int pos, int round, int n2) {
  // position 0 is fixed; positions 1..n2-1 rotate
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (n2 - 1);
}

__global__ __launch_bounds__(kJacobiThreads) void k_jacobi(double* As, double* ws, double* Vs, double* Vtmp_s,
                                                           int n) {
  double* A = As + (int64_t)blockIdx.x * n * n;
  double* V = Vtmp_s + (int64_t)blockIdx.x * n * n;
  double* Vout = Vs + (int64_t)blockIdx.x * n * n;
  double* w = ws + (int64_t)blockIdx.x * n;
  const int n2 = n + (n & 1);
  const int np = n2 / 2;
  __shared__ double cs[512], sn[512];
  __shared__ int pp[512], qq[512];
  __shared__ int rotated;
  __shared__ double fro;
  for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x) V[t] = (t % n == t / n) ? 1.0 : 0.0;
  // Frobenius norm for the absolute threshold (one wave, fixed order)
  if (threadIdx.x < 64) {
    double acc = 0.0;
    for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += 64) acc += A[t] * A[t];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (threadIdx.x == 0) fro = sqrt(acc);
  }
  __syncthreads();
  const double abs_tiny = fro * 1e-16 + 1e-300;
  for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < n2 - 1; ++round) {
      for (int k = threadIdx.x; k < np; k += blockDim.x) {
        int p = rr_player(k, round, n2), q = rr_player(n2 - 1 - k, round, n2);
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          double apq = A[p + (int64_t)q * n];
          double app = A[p + (int64_t)p * n], aqq = A[q + (int64_t)q * n];
          if (fabs(apq) > abs_tiny && fabs(apq) > 1e-15 * sqrt(fabs(app) * fabs(aqq))) {
            double tau = (aqq - app) / (2.0 * apq);
            double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rotated = 1;
          }
        }
        pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s;
      }
      __syncthreads();
      // rows p, q of A <- J^T A
      for (int64_t t = threadIdx.x; t < (int64_t)np * n; t += blockDim.x) {
        int k = (int)(t / n), col = (int)(t % n);
        double s = sn[k];
        if (s == 0.0) continue;
        double c = cs[k];
        int p = pp[k], q = qq[k];
        double ap = A[p + (int64_t)col * n], aq = A[q + (int64_t)col * n];
        A[p + (int64_t)col * n] = c * ap - s * aq;
        A[q + (int64_t)col * n] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of A <- A J and of V <- V J
      for (int64_t t = threadIdx.x; t < (int64_t)np * n; t += blockDim.x) {
        int k = (int)(t / n), row = (int)(t % n);
        double s = sn[k];
        if (s == 0.0) continue;
        double c = cs[k];
        int p = pp[k], q = qq[k];
        double ap = A[row + (int64_t)p * n], aq = A[row + (int64_t)q * n];
        A[row + (int64_t)p * n] = c * ap - s * aq;
        A[row + (int64_t)q * n] = s * ap + c * aq;
        double vp = V[row + (int64_t)p * n], vq = V[row + (int64_t)q * n];
        V[row + (int64_t)p * n] = c * vp - s * vq;
        V[row + (int64_t)q * n] = s * vp + c * vq;
      }
      __syncthreads();
    }
    const int any = rotated;   // read by every thread before thread 0 may reset it
    __syncthreads();
    if (!any) break;
  }
  // sort ascending (stable by index) and write out
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double wi = A[i + (int64_t)i * n];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      double wj = A[j + (int64_t)j * n];
      rank += (wj < wi) || (wj == wi && j < i);
    }
    w[rank] = wi;
    for (int r = 0; r < n; ++r) Vout[r + (int64_t)rank * n] = V[r + (int64_t)i * n];
  }
}

size_t syev_work_count(int n, int count) { return (size_t)n * n * count; }

int syev_batched(double* A, double* w, double* V, int n, int count, double* work, hipStream_t s) {
  if (n <= 0 || count <= 0) return RW_OK;
  RW_CHECK(n <= 1022, RW_EINVAL, "Jacobi eigensolver limited to n <= 1022 (got %d)", n);
  k_jacobi<<<count, kJacobiThreads, 0, s>>>(A, w, V, work, n);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// LU with partial pivoting and solve, one workgroup: A (n x n) and B (n x nrhs) column-major.
// Pivot search by wave 0 (ties -> lowest row).  stat[0] = min |pivot| / max |a_ij|, or 0 when a
// pivot falls below 1e-14 max |a_ij| (the solve is then abandoned).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_lu_solve(double* A, int n, double* B, int nrhs, double* stat) {
  __shared__ double s_amax, s_piv, s_minpiv;
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
        s_piv = best;
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

int lu_solve(double* A, int n, double* B, int nrhs, double* stat, hipStream_t s) {
  if (n <= 0) return RW_OK;
  k_lu_solve<<<1, 1024, 0, s>>>(A, n, B, nrhs, stat);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // namespace rw
