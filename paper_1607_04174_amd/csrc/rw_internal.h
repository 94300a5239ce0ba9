// Internal declarations shared by the librw translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/rw.h"

namespace rw {

// dynamic LDS budget of a workgroup (the kernels' static LDS stays below 64 bytes)
constexpr size_t kLdsLimit = 160 * 1024 - 64;

// Workgroup barrier that orders only LDS traffic: it does not wait for outstanding global stores
// (used where waves exchange data through LDS alone; global writes there are never read back
// inside the kernel).
// Cross-lane sums and maxima by DPP (VALU data movement: no LDS round trip per step).  dpp_mov<CTRL>
// moves a double across lanes by one DPP pattern; row16_* combine the 16 lanes of a DPP row (quad swaps,
// half-row mirror, row mirror), each step combining two equal partials in swapped order so that every
// lane of the row holds the same value; wave_* then combine the four rows in a fixed order through lane
// reads, giving every lane the same result.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double quad_sum(double x) {   // the 4 lanes of a quad
  x += dpp_mov<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_mov<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  return x;
}
__device__ __forceinline__ double row16_sum(double x) {
  x = quad_sum(x);
  x += dpp_mov<0x141>(x);   // row_half_mirror
  x += dpp_mov<0x140>(x);   // row_mirror
  return x;
}
__device__ __forceinline__ double row16_max(double x) {
  x = fmax(x, dpp_mov<0xB1>(x));
  x = fmax(x, dpp_mov<0x4E>(x));
  x = fmax(x, dpp_mov<0x141>(x));
  x = fmax(x, dpp_mov<0x140>(x));
  return x;
}
__device__ __forceinline__ double row16_min(double x) {
  x = fmin(x, dpp_mov<0xB1>(x));
  x = fmin(x, dpp_mov<0x4E>(x));
  x = fmin(x, dpp_mov<0x141>(x));
  x = fmin(x, dpp_mov<0x140>(x));
  return x;
}
__device__ __forceinline__ double lane_read(double x, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double wave_sum64(double x) {
  x = row16_sum(x);
  return (lane_read(x, 0) + lane_read(x, 16)) + (lane_read(x, 32) + lane_read(x, 48));
}
__device__ __forceinline__ double wave_max64(double x) {
  x = row16_max(x);
  return fmax(fmax(lane_read(x, 0), lane_read(x, 16)), fmax(lane_read(x, 32), lane_read(x, 48)));
}
__device__ __forceinline__ double wave_min64(double x) {
  x = row16_min(x);
  return fmin(fmin(lane_read(x, 0), lane_read(x, 16)), fmin(lane_read(x, 32), lane_read(x, 48)));
}

// lane U of each row of 16 lanes, in every lane of that row (64-bit DPP row broadcast)
template <int U>
__device__ __forceinline__ double row_bcast(double x) {
  return __builtin_amdgcn_update_dpp(0.0, x, 0x150 + U, 0xF, 0xF, true);
}

// f(integral_constant<int, I>) for I = B .. E-1, in order
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---- error reporting ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
// Pinned host buffer of at least `bytes` for small device-to-host reads, one per host thread (grown on demand,
// held until the process ends).  Reads into pageable memory wait for each copy in turn; reads into this buffer
// are queued on the stream and waited for once.  The contents are the caller's until its next call.
int host_stage(size_t bytes, void** p);

#define RW_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      ::rw::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return RW_EHIP;                                                                       \
    }                                                                                       \
  } while (0)

#define RW_CHECK(cond, code, ...)      \
  do {                                 \
    if (!(cond)) {                     \
      ::rw::set_error(__VA_ARGS__);    \
      return (code);                   \
    }                                  \
  } while (0)

#define RW_TRY(expr)              \
  do {                            \
    int s_ = (expr);              \
    if (s_ != RW_OK) return s_;   \
  } while (0)

#define RW_LAUNCH_CHECK() RW_HIP(hipGetLastError())

// Synchronous entry points wait for their stream or read device values on the host, which a stream under
// HIP graph capture cannot do: they refuse such a stream up front (nothing is enqueued).
#define RW_NOT_CAPTURING(stream)                                                                      \
  do {                                                                                                 \
    hipStreamCaptureStatus cs_ = hipStreamCaptureStatusNone;                                         \
    RW_HIP(hipStreamIsCapturing((stream), &cs_));                                                      \
    RW_CHECK(cs_ == hipStreamCaptureStatusNone, RW_ECAPTURE,                                         \
             "%s waits for its stream; under HIP graph capture use the RW_ASYNC entry points", __func__); \
  } while (0)

// ---- workspace carving -------------------------------------------------------------------------
// A bump allocator over a caller-owned device buffer; every block is 256-byte aligned.  With a null
// base it only measures.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

inline size_t dtype_size(int dt) { return dt == RW_F64 ? 8 : (dt == RW_F32 ? 4 : 2); }
// eigenbasis storage: the plain types, or the BF16 pair form (remainder columns of q_1 .. q_kPairCols, then
// the plain BF16 block)
constexpr int kPairCols = RW_PAIR_COLS;
inline bool q_dtype_ok(int dt) { return dt == RW_F64 || dt == RW_F32 || dt == RW_BF16 || dt == RW_BF16_PAIR; }
inline int64_t q_block_cols(int dt, int64_t m) { return dt == RW_BF16_PAIR ? m + kPairCols : m; }
// a basis as its plain block (element type dt) and, for the pair form, the remainder columns (else null)
struct BasisView {
  const void* hi;
  const uint16_t* lo;
  int dt;
};
inline BasisView basis_view(int64_t N, const void* Q, int qdt) {
  if (qdt == RW_BF16_PAIR)
    return {static_cast<const uint16_t*>(Q) + (int64_t)kPairCols * N, static_cast<const uint16_t*>(Q), RW_BF16};
  return {Q, nullptr, qdt};
}

// ---- the graph handle --------------------------------------------------------------------------
struct Graph {
  int ndim = 2;
  int64_t nx = 1, ny = 1, nz = 1, N = 0;
  int conn = 4, ndir = 2;
  int dtype = RW_F64;
  int weight_form = RW_WEIGHT_SQUARED;
  int normalized = 1;
  double beta = 0.0;
  int dx[4] = {0, 0, 0, 0}, dy[4] = {0, 0, 0, 0}, dz[4] = {0, 0, 0, 0};
  int64_t off[4] = {0, 0, 0, 0};
  // device arrays inside the caller's graph buffer
  double* J = nullptr;      // N
  double* scale = nullptr;  // ndir x N (FP64 on every graph)
  double* weight = nullptr; // ndir x N (FP64 on every graph)
  void* coef = nullptr;     // ndir x N (dtype)
  void* diag = nullptr;     // N (dtype)
  void* dinv = nullptr;     // N (dtype)
  void* ghat = nullptr;     // N (dtype)
  double* degree = nullptr; // N
  uint8_t* mask = nullptr;  // N
  std::vector<uint8_t> hmask;   // host copy of mask (empty until the first edit reads it; only edits change it)
  double* partial = nullptr;  // reduction partials (kReduceBlocks)
  double* sums = nullptr;     // [0] = sum of degrees
  int64_t* comp = nullptr;    // N: component root (the smallest node index) over edges with w >= kAnchorWeight
  int* cc_flag = nullptr;     // device scratch for the component and anchoring kernels
  bool cc_valid = false;      // comp matches the current weights
  bool cc_recheck = false;    // comp matched the weights before the last rebuilds: still valid unless an edge
                              // crossed kAnchorWeight since (device flag cc_flag[4], set by the weight kernel)
};

// edges below this weight do not connect nodes for the solvability check (they underflow in FP32)
constexpr double kAnchorWeight = 1e-30;

constexpr int kReduceBlocks = 1024;

// kernel-side copy of the grid geometry
struct GridDev {
  int64_t nx, ny, nz, N;
  int ndir;
  int dx[4], dy[4], dz[4];
  int64_t off[4];
};

inline GridDev grid_of(const Graph* g) {
  GridDev d;
  d.nx = g->nx; d.ny = g->ny; d.nz = g->nz; d.N = g->N; d.ndir = g->ndir;
  for (int k = 0; k < 4; ++k) {
    d.dx[k] = g->dx[k]; d.dy[k] = g->dy[k]; d.dz[k] = g->dz[k]; d.off[k] = g->off[k];
  }
  return d;
}

// is the head (x,y,z) + dir inside the grid?
__device__ __forceinline__ bool head_in(const GridDev& G, int64_t x, int64_t y, int64_t z, int d) {
  int64_t a = x + G.dx[d], b = y + G.dy[d], c = z + G.dz[d];
  return a >= 0 && a < G.nx && b >= 0 && b < G.ny && c >= 0 && c < G.nz;
}
// is the tail (x,y,z) - dir inside the grid?
__device__ __forceinline__ bool tail_in(const GridDev& G, int64_t x, int64_t y, int64_t z, int d) {
  int64_t a = x - G.dx[d], b = y - G.dy[d], c = z - G.dz[d];
  return a >= 0 && a < G.nx && b >= 0 && b < G.ny && c >= 0 && c < G.nz;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// bf16 storage helpers (round-to-nearest-even on store)
__device__ __forceinline__ float bf16_to_f32(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// typed element access for the three storage types
template <typename T> struct Elem;
template <> struct Elem<double> {
  using C = double;  // compute type
  __device__ static double ld(const double* p, int64_t i) { return p[i]; }
  __device__ static void st(double* p, int64_t i, double v) { p[i] = v; }
};
template <> struct Elem<float> {
  using C = float;
  __device__ static float ld(const float* p, int64_t i) { return p[i]; }
  __device__ static void st(float* p, int64_t i, float v) { p[i] = v; }
};
template <> struct Elem<uint16_t> {
  using C = float;
  __device__ static float ld(const uint16_t* p, int64_t i) { return bf16_to_f32(p[i]); }
  __device__ static void st(uint16_t* p, int64_t i, float v) { p[i] = f32_to_bf16(v); }
};

size_t graph_layout(const rw_graph_desc& d, Graph* g, void* buf);  // returns bytes
int graph_rebuild(Graph* g, hipStream_t s);   // weights -> degree, dinv, ghat, coef, diag
// Connected components of the graph restricted to edges with w >= kAnchorWeight (computed on first use
// after a build or edit, then cached), and the check that every component holds a seed: RW_EUNANCHORED
// otherwise.  seeds: device array of S node ids; flags: device scratch of N bytes.
int graph_components(Graph* g, hipStream_t s);
int check_anchored(Graph* g, const int64_t* seeds, int64_t S, uint8_t* flags, hipStream_t s);
// the same check queued on the stream without waiting: *bad_dev is the device int that is nonzero when some
// component holds no seed, valid once the stream reaches this point (kept until the next components call)
int anchor_launch(Graph* g, const int64_t* seeds, int64_t S, uint8_t* flags, hipStream_t s, const int** bad_dev);
// The anchoring check with kernels only (no memset, no host read; capturable): needs the components current
// (g->cc_valid, e.g. after rw_graph_components); *bad_dev (device int) ends 1 when a component holds no seed.
int anchor_launch_async(const Graph* g, const int64_t* seeds, int64_t S, uint8_t* flags, int* bad_dev, hipStream_t s);
// fill kernels (capturable in place of hipMemsetAsync)
int fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
int fill_i32(int* p, int64_t n, int v, hipStream_t s);

// ---- stencil operator --------------------------------------------------------------------------
// Y = alpha * op(X) + beta * X + gamma * Z   (column-major N x b, graph dtype)
int stencil_apply(const Graph* g, const void* X, void* Y, const void* Z, int64_t b, double alpha,
                  double beta, double gamma, hipStream_t s,
                  hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

// ---- tall-skinny dense kernels (blas.hip) -------------------------------------------------------
// G (FP64, bx x by, column-major, ld = bx) = X^T Y for column-major X (rows x bx, ld ldx) and
// Y (rows x by, ld ldy) of element type dt (RW_F64 / RW_F32 / RW_BF16).  Deterministic two-stage
// reduction over row chunks through `partial` (gram_partial_count doubles).
size_t gram_partial_count(int64_t rows, int bx, int by);
// sym: the product is known to be symmetric (X = Y, or X^T M X with M symmetric); only the upper tiles
// are computed and mirrored.  acc32 (FP32 blocks with sym only): chunks of rows may accumulate in FP32,
// an error near FP32's unit roundoff times the column norms; for nearly orthonormal blocks only (an
// ill-conditioned Gram needs the FP64 accumulation).
int gram(int dt, const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t rows, int bx, int by,
         double* G, double* partial, hipStream_t s, bool sym = false, bool acc32 = false);
// Z (rows x n, ld ldz, type dt) = X (rows x k, ld ldx, type dt) * V (FP64, k x n, ld ldv)
//   (+ beta * Z when beta != 0)
int gemm_tn(int dt, const void* X, int64_t ldx, const double* V, int64_t ldv, void* Z, int64_t ldz,
            int64_t rows, int k, int n, double beta, hipStream_t s);
// true when gemm_tn with these sizes runs the single-slab matrix-core kernel, in which each 32-row task
// reads all of its rows of X before it writes its rows of Z: Z may then share X's storage (same leading
// dimension, shifted by whole columns), an in-place rotation
bool gemm_rowwise(int dt, int64_t rows, int k, int n);
// X = A0 V, LX = A1' V and res_j = ||LX_j - theta_j X_j|| in one pass for FP32 blocks (rows x k inputs with
// leading dimension ld, V FP64 k x n); A1' is A1 (k - off1 columns) behind off1 zero columns.  LX may be
// null (op X is then not stored, only its residual norms formed).  X may share
// A0's storage shifted by whole columns.  rotate_pair_fits tells whether the shape is supported; `partial`
// holds rotate_pair_partial_count(n) doubles.
bool rotate_pair_fits(int dt, int64_t rows, int k, int n);
size_t rotate_pair_partial_count(int n);
int rotate_pair(const float* A0, const float* A1, int off1, int64_t ld, const double* V, int64_t ldv,
                const double* theta, float* X, float* LX, int64_t rows, int k, int n, double* res, double* partial,
                hipStream_t s);
// copy / convert a column-major block (rows x cols) between element types
int convert_block(int dt_src, const void* src, int64_t lds, int dt_dst, void* dst, int64_t ldd,
                  int64_t rows, int cols, hipStream_t s);
// the BF16 pair form (rows x (kPairCols + cols)) of an F64 / F32 block
int convert_pair(int dt_src, const void* src, int64_t rows, uint16_t* dst, int cols, hipStream_t s);
// P = Q^T X (m x C FP64, leading dimension m) for a basis of any storage type: X is F64 for an F64 basis, F32
// otherwise (C x N label-major); F64 / F32 bases by FP64-accumulated VALU products, BF16 and the pair form on
// the matrix cores (the pair form's remainder columns add to rows 1 .. 8).  partial: project_block_partial_bytes;
// tmp: 8 C doubles (pair form only).
size_t project_block_partial_bytes(int64_t N, int m, int C);
// the VALU projection of F64 / F32 bases behind project_block (FP64 accumulation, fixed-order chunk sums)
size_t project_cols_partial_count(int64_t N, int m, int C);
int project_cols(int dt, const void* Q, int64_t N, int m, const void* X, int C, double* P, double* partial,
                 hipStream_t s);
int project_block(const void* Q, int qdt, int64_t N, int m, const void* X, int C, double* P, void* partial,
                  double* tmp, hipStream_t s);
// column norms (FP64 out) of R = A - B diag(theta) (theta may be null: plain norms of A)
size_t norm_partial_count(int cols);
int residual_norms(int dt, const void* A, const void* B, const double* theta, int64_t rows, int cols,
                   int64_t ld, double* out, double* partial, hipStream_t s);
// d_j = a_j^T b_j (FP64) for column-major A, B (rows x cols, ld)
int col_dots(int dt, const void* A, const void* B, int64_t rows, int cols, int64_t ld, double* out,
             double* partial, hipStream_t s);
// out[0] = max_i |x_i|
int absmax(const double* x, int64_t n, double* out, hipStream_t s);
// fill a block with deterministic pseudo-random normals (counter-based: splitmix64 + Box-Muller)
int fill_random(int dt, void* X, int64_t ld, int64_t rows, int cols, uint64_t seed, hipStream_t s);
// X -= v (v^T X) for a unit vector v (rows), X column-major rows x cols
int project_out(int dt, void* X, int64_t ld, const void* v, int64_t rows, int cols, double* tmp,
                double* partial, hipStream_t s);
// Y = X - v (v^T X), reading X and writing Y (Y may be X)
int project_out_to(int dt, const void* X, int64_t ldx, void* Y, int64_t ldy, const void* v, int64_t rows, int cols,
                   double* tmp, double* partial, hipStream_t s);

// ---- BF16 matrix-core contractions (mfma.hip) ----------------------------------------------------
// U = s_i sum_{j>=1} Q(i, j) Y(j, c) + kappa_c on non-seeds (s = d^{-1/2} or 1; kappa_c = Y(0, c), added
// where s > 0 or the operator is L), one-hot on seeds; Y is m x C (ld m) in the form k_solve_coeffs leaves
int reconstruct_mfma(const Graph* g, const void* Q, const uint16_t* Qlo, int m, const double* Y, int C,
                     const uint8_t* map, void* U, hipStream_t s);

// ---- FP64 view of the operator and of a stored basis, for the online solve (solve.hip) ------------
// Seed rows of the reduced system are formed from the FP64 weights and degrees (the graph's type only
// rounds the stencil's coefficients), and the stored basis is taken as the exact FP64 null vector plus
// the other columns made orthogonal to it in FP64:
//   q'_0 = g,   q'_j = (q_j - g c_j) / n_j,   c_j = g^T q_j,   n_j = ||q_j - g c_j||   (j >= 1).
// In a weakly coupled graph the reduced system has condition numbers near 1/u, and the rounding of an
// FP32 coefficient or of a stored low-precision null vector would decide its solution.
__device__ __forceinline__ double dinv64(const double* degree, int64_t x) {
  const double d = degree[x];
  return d > 0.0 ? 1.0 / sqrt(d) : 0.0;
}
// unit null vector in FP64: D^{1/2} 1 / ||D^{1/2} 1|| (sums[0] = 1^T D 1) or 1 / sqrt(N)
__device__ __forceinline__ double ghat64(const double* degree, const double* sums, int normalized, int64_t N,
                                         int64_t x) {
  return normalized ? sqrt(degree[x]) / sqrt(sums[0]) : 1.0 / sqrt((double)N);
}
// s_i g_i on a node with d_i > 0 (s = d^{-1/2} or 1): the same for every node
__device__ __forceinline__ double ghat_scaled64(const double* sums, int normalized, int64_t N) {
  return normalized ? 1.0 / sqrt(sums[0]) : 1.0 / sqrt((double)N);
}
// cn[j] = c_j and cn[m + j] = n_j for j in [1, m) (cn[0] = 0, cn[m] = 1) of the column-major N x m basis Q
// (column 0 the null vector); *bad (device) is set when some n_j is not positive.  partial holds
// null_stats_partial_count(N, m) doubles.
size_t null_stats_partial_count(int64_t N, int m);
int null_stats(const Graph* g, const void* Q, int qdt, int m, double* partial, double* cn, int* bad, hipStream_t s);
// U = s * sum_{j>=1} q_j Y_j + kappa (one-hot on the nodes map marks) for C labels of the solve's Y (m x C, after
// solve_coeffs), U of the graph's dtype (solve.hip)
int reconstruct_any(const Graph* g, const void* Q, int qdt, int m, const double* Y, int C, const uint8_t* map,
                    void* U, hipStream_t s);
// After the reduced solve (Y, m x C, ld m, the coefficients of the q'_j), in place and by one workgroup:
// Y(j, c) /= n_j for j >= 1, then Y(0, c) = kappa_c = sg (Y(0, c) - sum_{j>=1} c_j Y(j, c)) with
// sg = ghat_scaled64, so that U = s_i sum_{j>=1} q_j(i) Y(j, c) + kappa_c on nodes with s_i > 0.
// The column sums run in order in one lane per label.
__device__ __forceinline__ void solve_coeffs_block(double* Y, int m, int C, const double* cn, double sg) {
  for (int64_t t = threadIdx.x; t < (int64_t)m * C; t += blockDim.x) {
    const int j = (int)(t % m);
    if (j > 0) Y[t] /= cn[m + j];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    double* y = Y + (int64_t)c * m;
    double acc = y[0];
    for (int j = 1; j < m; ++j) acc -= cn[j] * y[j];
    y[0] = sg * acc;
  }
}
// launch of solve_coeffs_block for one system (solve.hip)
int solve_coeffs(double* Y, int m, int C, const double* cn, const Graph* g, hipStream_t s);


// The reduced system from the seed rows (leading dimension ld, S seeds): K(i, j) = (lambda_i + gamma) [i == j]
// - sum_s Qs(s, i) GB(s, j) for j < m, Y(i, c) = sum_s Qs(s, i) Hs(s, c) for c < C; each entry sums its S
// products in seed order (the single and the batched solves form the system with this same code).  A 32 x 32
// tile of the m x (m + C) output per 256-thread workgroup (tile (bx, by): rows 32 bx.., columns 32 by..;
// thread (ty, tx) the entries (32 bx + ty + 16 a, 32 by + tx + 16 b)), the seed rows staged in LDS 32 at a time.
// sA, sB: 32 x 33 doubles each in LDS.
constexpr int kRedTile = 32;
__device__ __forceinline__ void reduced_tile(int bx, int by, int m, int C, int64_t S, int64_t ld, const double* Qs,
                                             const double* GB, const double* Hs, const double* lambda,
                                             double gamma, double* K, double* Y, double* sA, double* sB) {
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = kRedTile * bx, j0 = kRedTile * by;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t s0 = 0; s0 < S; s0 += kRedTile) {
    // columns of the tile: 32 seeds each, consecutive threads on consecutive seeds
    for (int e = tid; e < kRedTile * kRedTile; e += 256) {
      const int q = e & 31, c = e >> 5;
      const int64_t s = s0 + q;
      const int i = i0 + c, j = j0 + c;
      sA[q * 33 + c] = (s < S && i < m) ? Qs[s + (int64_t)i * ld] : 0.0;
      const double* bc = j < m ? GB + (int64_t)j * ld : Hs + (int64_t)(j - m) * ld;
      sB[q * 33 + c] = (s < S && j < m + C) ? bc[s] : 0.0;
    }
    __syncthreads();
    const int nq = (int)(S - s0 < kRedTile ? S - s0 : kRedTile);
    for (int q = 0; q < nq; ++q) {
      const double a0 = sA[q * 33 + ty], a1 = sA[q * 33 + ty + 16];
      const double b0 = sB[q * 33 + tx], b1 = sB[q * 33 + tx + 16];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = i0 + ty + 16 * a, j = j0 + tx + 16 * b;
      if (i >= m || j >= m + C) continue;
      if (j < m) K[i + (int64_t)j * m] = (i == j ? lambda[i] + gamma : 0.0) - acc[a][b];
      else Y[i + (int64_t)(j - m) * m] = acc[a][b];
    }
}

// Seed row k (node i, leading dimension ld) of the reduced system's inputs, formed by one workgroup from
// the FP64 weights and degrees: for j < m, Qs(k, j) = q'_j(i) and GB(k, j) = (B q'_j)(i) = -sum over the
// non-seed neighbours t of coef(i, t) q'_j(t), with coef(i, t) = w_it d_i^{-1/2} d_t^{-1/2} (or w_it);
// for c < C, Us(k, c) = U_hat(i, c) (d_i^{1/2} or 1 on the seed's label) and Hs(k, c) = (op_ss U_hat_s)(i, c).
// With cn == nullptr the stored columns q_j are gathered as they are and g(i), (B g_n)(i) go to gs[k],
// Bg[k] for a later correction (the choice of m fits the stored columns); otherwise the q'_j of cn.
template <typename TQ>
__device__ void gather_seed_row(const GridDev& G, int normalized, const double* weight, const double* degree,
                                const double* sums, const TQ* Q, const TQ* Qlo, int m, const uint8_t* map,
                                int64_t i, int C,
                                const double* cn, int64_t k, int64_t ld, double* Qs, double* GB, double* Hs,
                                double* Us, double* gs, double* Bg) {
  const int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / (G.nx * G.ny);
  const double di = normalized ? dinv64(degree, i) : 1.0;
  int64_t nb[8];
  double cf[8];
  int cnt = 0;
  for (int d = 0; d < G.ndir; ++d) {
    if (head_in(G, x, y, z, d)) {
      const int64_t t = i + G.off[d];
      const double w = weight[d * G.N + i];
      nb[cnt] = t;
      cf[cnt++] = normalized ? w * di * dinv64(degree, t) : w;
    }
    if (tail_in(G, x, y, z, d)) {
      const int64_t t = i - G.off[d];
      const double w = weight[d * G.N + t];
      nb[cnt] = t;
      cf[cnt++] = normalized ? w * di * dinv64(degree, t) : w;
    }
  }
  // g(i) and (B g_n)(i)
  const double gi = ghat64(degree, sums, normalized, G.N, i);
  double bg = 0.0;
  for (int t = 0; t < cnt; ++t)
    if (map[nb[t]] == 0) bg -= cf[t] * ghat64(degree, sums, normalized, G.N, nb[t]);
  // Qlo (the pair form's remainder columns, or null): column j in [1, kPairCols] is read as hi + lo, exact in
  // FP64
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const TQ* qc = Q + (int64_t)j * G.N;
    const TQ* lc = (Qlo != nullptr && j >= 1 && j <= kPairCols) ? Qlo + (int64_t)(j - 1) * G.N : nullptr;
    double qv = (double)Elem<TQ>::ld(qc, i);
    if (lc) qv += (double)Elem<TQ>::ld(lc, i);
    double acc = 0.0;
    for (int t = 0; t < cnt; ++t)
      if (map[nb[t]] == 0) {
        double v = (double)Elem<TQ>::ld(qc, nb[t]);
        if (lc) v += (double)Elem<TQ>::ld(lc, nb[t]);
        acc -= cf[t] * v;
      }
    if (cn != nullptr) {
      if (j == 0) {
        qv = gi;
        acc = bg;
      } else {
        qv = (qv - gi * cn[j]) / cn[m + j];
        acc = (acc - bg * cn[j]) / cn[m + j];
      }
    }
    Qs[k + (int64_t)j * ld] = qv;
    GB[k + (int64_t)j * ld] = acc;
  }
  if (cn == nullptr && threadIdx.x == 0) {
    gs[k] = gi;
    Bg[k] = bg;
  }
  const double diag = normalized ? (degree[i] > 0.0 ? 1.0 : 0.0) : degree[i];
  for (int lab = threadIdx.x; lab < C; lab += blockDim.x) {
    auto uhat = [&](int64_t node, int mlab) -> double {
      if (mlab - 1 != lab) return 0.0;
      return normalized ? sqrt(degree[node]) : 1.0;
    };
    const double own = uhat(i, map[i]);
    double acc = diag * own;
    for (int t = 0; t < cnt; ++t) {
      const int ml = map[nb[t]];
      if (ml != 0) acc -= cf[t] * uhat(nb[t], ml);
    }
    Hs[k + (int64_t)lab * ld] = acc;
    Us[k + (int64_t)lab * ld] = own;
  }
}

// ---- small dense FP64 kernels, one workgroup per matrix (dense.hip) ------------------------------
// In-place lower Cholesky of count matrices (n x n, ld n, stride n*n); info[b] = 0 or (k+1) of the
// first non-positive pivot.
int chol_batched(double* A, int n, int count, int* info, hipStream_t s);
// Rinv = (L^T)^{-1} (upper triangular) for the lower factor L; n x n
int chol_upper_inverse(const double* L, double* Rinv, int n, hipStream_t s);
// W = (L^T)^{-1} for the Cholesky factor of G (n x n, lower triangle read; G may be overwritten);
// info[0] = k + 1 at the first failed pivot (W then undefined), else 0.
int chol_inverse(double* G, double* W, int n, int* info, hipStream_t s);
// Symmetric eigendecomposition (parallel cyclic Jacobi) of count matrices A (n x n, stride n*n, read
// only): w (ascending, stride n); V (n x n eigenvectors, or null); R (n x nrhs per matrix, or null)
// is replaced by V^T R.  work: syev_work_count doubles.  min_rel_tol raises the relative rotation
// threshold (|a_pq| against sqrt(|a_pp a_qq|)) above its FP64 default, for matrices whose entries carry
// larger errors than FP64 rounding (0: the default).
int syev_batched(const double* A, double* w, double* V, double* R, int nrhs, int n, int count, double* work,
                 hipStream_t s, double min_rel_tol = 0.0);
size_t syev_work_count(int n, int count, bool vectors, int nrhs);
// Symmetric eigendecomposition of one matrix (3 <= n <= 256) through its tridiagonal form; returns
// RW_ENOCONV without an error message when eigenvalues are too close for inverse iteration.
// tridiag_batch_fits: the orders the batched solver takes (3 <= n <= 199, the reduction wholly in LDS).
bool tridiag_fits(int n);
bool tridiag_batch_fits(int n);
size_t tridiag_work_count(int n);
// With flag_dev, nothing waits: the call returns RW_OK and *flag_dev is the device double that is nonzero
// where the result is RW_ENOCONV (then V is not valid).
int syev_tridiag(const double* A, double* w, double* V, int n, double* work, hipStream_t s,
                 const double** flag_dev = nullptr);
// Batched eigenvalues and rotated right-hand sides through the tridiagonal form, for the candidate problems
// of the choice of m: matrix b (order sizes[b] <= ld, leading dimension ld, ld^2 apart) has right-hand
// sides R_b (ld x C, ld * C apart); on RW_OK, w_b holds its eigenvalues (zero beyond sizes[b]) and
// R_b = V_b^T R_b (zero rows beyond sizes[b]).  RW_ENOCONV (clustered eigenvalues) leaves w and R as they
// were.  work holds tridiag_rhs_work_count(max size, count, C) doubles.  With flag_dev, nothing waits: the
// call returns RW_OK and *flag_dev is the device double that is nonzero where the result is RW_ENOCONV.
constexpr int kTriBatchMax = 32;
struct TriSizes {
  int n[kTriBatchMax];
};
size_t tridiag_rhs_work_count(int nmax, int count, int C);
int syev_tridiag_rhs(const double* A, int ld, const int* sizes, int count, double* R, int C, double* w, double* work,
                     size_t work_count, hipStream_t s, const double** flag_dev = nullptr);
// Solve A X = B by LU with partial pivoting (A: n x n, B: n x nrhs, both destroyed/overwritten;
// X returned in B).  stat[0] = min |pivot| / max |a_ij| (0 if a pivot is below the threshold).
int lu_solve(double* A, int n, double* B, int nrhs, double* stat, hipStream_t s);
struct LuJob {
  double* A;
  double* B;
  double* stat;
  int n;
  int nrhs;
};
// one LU solve per job (jobs in device memory)
int lu_solve_batched(const LuJob* jobs, int count, hipStream_t s);

}  // namespace rw

struct rw_graph_s {
  rw::Graph g;
};
