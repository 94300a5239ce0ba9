// The walker driven by priors alone, at registration label counts (thousands of displacement labels).
// Sec. II-A eq. (5) with the seed set empty: (L + gamma I) U = gamma P on every vertex; under the normalized
// Laplacian in hat variables (Sec. II-C), (L_hat + gamma I) U_hat = gamma P_hat with U_hat = D^{1/2} U and
// P_hat = D^{1/2} P.  Sec. II-B eq. (15) with no seed rows gives U_hat = Q' (Lambda + gamma I)^{-1} gamma
// Q'^T P_hat on the FP64 basis Q' = [g, (q_j - g c_j) / n_j] of the seeded solves (the null vector exact).
// Sec. III-A2 eq. (25): m from g_k(m) on one label in every r^d.  The registration result is, per voxel,
// the label of largest probability (its displacement) and that probability.
//
//   projection    Z_hat = Q^T P_hat over the stored columns, and g^T P_hat (one read of P).  On a BF16 basis
//                 on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 within a voxel chunk, FP64 over the
//                 chunks), D^{1/2} folded into the staged Q tile so that the priors enter as stored, and g
//                 as one more staged column;
//   choice of m   ||p_hat_k||^2 on the sampled labels and the prefix sums of Z_hat (host);
//   coefficients  Z' = Q'^T P_hat from Z_hat, g^T P_hat, c_j and n_j; Y = gamma (Lambda + gamma I)^{-1} Z',
//                 rescaled so that U = s * sum_{j>=1} q_j Y_j + kappa (s = D^{-1/2});
//   labels        the reconstruction fused with the arg max over the labels, U never written: on a BF16
//                 basis the matrix cores over a voxel-major copy of the basis (one transposition per call)
//                 with kappa folded in against a last column holding s^{-1} = d^{1/2}; otherwise one thread
//                 per voxel;
//   U             optionally, the seeded solves' reconstruction.
#include <cmath>
#include <cstring>
#include <vector>

#include "rw_internal.h"

namespace rw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_bf16(uint4 a, uint4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// kappa of the label rows past C in the fused reconstruction: far below any probability, so they never win
constexpr float kPadKappa = -1e30f;

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  return (uint32_t)f32_to_bf16(lo) | ((uint32_t)f32_to_bf16(hi) << 16);
}

// ---------------------------------------------------------------------------------------------
// per-voxel scales: sv = s_i = d_i^{1/2} (1 under L), sg = s_i g_i, inv = 1 / s_i (0 where d_i = 0)
// ---------------------------------------------------------------------------------------------
__global__ void k_rwir_scales(const double* degree, const double* sums, int normalized, int64_t N, float* sv,
                              float* sg, float* inv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double s = normalized ? sqrt(degree[i]) : 1.0;
  sv[i] = (float)s;
  sg[i] = (float)(s * ghat64(degree, sums, normalized, N, i));
  inv[i] = s > 0.0 ? (float)(1.0 / s) : 0.0f;
}

// Qs[c Np + i] = BF16(s_i q_c(i)) for c < ma, BF16(s_i g_i) for c = ma, 0 for c in (ma, KC) and for i >= N;
// one thread per 8 voxels of one column (16-byte stores)
__global__ void k_rwir_scaled_basis(const uint16_t* __restrict__ Q, int ma, int64_t N, int64_t Np, int KC,
                                    const float* __restrict__ sv, const float* __restrict__ sg,
                                    uint16_t* __restrict__ Qs) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t per = Np / 8;
  if (t >= per * KC) return;
  const int c = (int)(t / per);
  const int64_t v = 8 * (t % per);
  float x[8];
  if (c > ma) {
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = 0.0f;
  } else if ((N & 7) == 0 && v + 8 <= N) {   // 16-byte rows: vector loads
    const float4 s0 = *reinterpret_cast<const float4*>((c < ma ? sv : sg) + v);
    const float4 s1 = *reinterpret_cast<const float4*>((c < ma ? sv : sg) + v + 4);
    const float sc[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
    if (c < ma) {
      const uint4 q = *reinterpret_cast<const uint4*>(Q + (int64_t)c * N + v);
      const uint32_t a[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[2 * u] = bf16_to_f32((uint16_t)(a[u] & 0xffffu)) * sc[2 * u];
        x[2 * u + 1] = bf16_to_f32((uint16_t)(a[u] >> 16)) * sc[2 * u + 1];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = sc[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t i = v + e;
      x[e] = i >= N ? 0.0f : (c < ma ? bf16_to_f32(Q[(int64_t)c * N + i]) * sv[i] : sg[i]);
    }
  }
  *reinterpret_cast<uint4*>(Qs + (int64_t)c * Np + v) =
      uint4{pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3]), pack_bf16(x[4], x[5]), pack_bf16(x[6], x[7])};
}

// ---------------------------------------------------------------------------------------------
// projection on the matrix cores (BF16 basis)
// ---------------------------------------------------------------------------------------------
// Workgroup: 8 waves, 256 labels x KC = 32 NH columns of the scaled basis Qs (s_i q_j(i) for the ma stored
// columns, s_i g_i, zeros: one pass per call, row stride Np), one chunk of voxels in stages of 64 (two K steps
// of 32).  Wave w takes labels 64 (w % 4) .. +63 (4 sub-tiles of 16) against column half w / 4 (NH tiles of 16),
// so that two waves share each SIMD.  The stage's Qs tile is copied to LDS ([column][voxel], padded row,
// double-buffered); the priors' fragments come from HBM straight into registers, one stage ahead (the two
// column halves read the same fragments; the second read hits the cache).  Output: FP32 partials per chunk,
// part[(chunk C + label) KC + column].  Measured at 96^3 x 3969 labels: 2.8 ms, 2.5 TB/s of priors.  Each label
// row contributes 128 contiguous bytes per stage, so HBM serves many short scattered pieces; four waves with
// all 224 columns each and two stages of priors in flight (three register sets) took 3.75 ms with the same
// partials, so the depth of prefetch is not what limits it.
constexpr int kPjVox = 64;
constexpr int kPjRow = kPjVox + 8;   // staged row in BF16 elements: conflict-free 16-byte fragment reads
constexpr int kPjLab = 256;
constexpr int kPjThreads = 512;

size_t rwir_proj_lds(int kc) { return (size_t)2 * kc * kPjRow * sizeof(uint16_t); }

template <typename TP>
__device__ __forceinline__ uint4 load_p8(const TP* row, int64_t v, int64_t vend, bool ok, bool vec);

template <>
__device__ __forceinline__ uint4 load_p8<uint16_t>(const uint16_t* row, int64_t v, int64_t vend, bool ok,
                                                   bool vec) {
  if (ok && vec && v + 8 <= vend) return *reinterpret_cast<const uint4*>(row + v);
  uint16_t e[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) e[q] = (ok && v + q < vend) ? row[v + q] : (uint16_t)0;
  return uint4{e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16), e[4] | ((uint32_t)e[5] << 16),
               e[6] | ((uint32_t)e[7] << 16)};
}

template <>
__device__ __forceinline__ uint4 load_p8<float>(const float* row, int64_t v, int64_t vend, bool ok, bool vec) {
  float e[8];
  if (ok && vec && v + 8 <= vend) {
    const float4 a = *reinterpret_cast<const float4*>(row + v), b = *reinterpret_cast<const float4*>(row + v + 4);
    e[0] = a.x; e[1] = a.y; e[2] = a.z; e[3] = a.w; e[4] = b.x; e[5] = b.y; e[6] = b.z; e[7] = b.w;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = (ok && v + q < vend) ? row[v + q] : 0.0f;
  }
  return uint4{pack_bf16(e[0], e[1]), pack_bf16(e[2], e[3]), pack_bf16(e[4], e[5]), pack_bf16(e[6], e[7])};
}

template <typename TP, int NH, bool VEC>
__global__ __launch_bounds__(kPjThreads) void k_rwir_proj(const uint16_t* __restrict__ Qs, int64_t Np, int64_t N,
                                                          const TP* __restrict__ P, int C, int64_t chunk, int nlt,
                                                          int64_t nwg, float* __restrict__ part) {
  constexpr int KC = 32 * NH;
  constexpr int PIECES = KC * (kPjVox / 8);            // 16-byte pieces of one staged tile
  constexpr int PQ = (PIECES + kPjThreads - 1) / kPjThreads;
  extern __shared__ __align__(16) char smem[];
  uint16_t* sQ = reinterpret_cast<uint16_t*>(smem);   // [2][KC][kPjRow]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lg = wave & 3, c0 = (wave >> 2) * NH;      // label group, first column tile
  // XCD-contiguous workgroups: the label tiles of one voxel chunk run on one XCD and share its L2
  const int64_t per_xcd = (nwg + 7) / 8;
  const int64_t L = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (L >= nwg) return;
  const int64_t ck = L / nlt;
  const int lt = (int)(L % nlt);
  const int64_t vb = ck * chunk, ve = min(N, vb + chunk);
  const int nst = (int)((ve - vb + kPjVox - 1) / kPjVox);
  // VEC (16-byte rows): the full stages run without checks and the chunk's partial last stage, if any, after
  // them with checks; otherwise every stage checks
  const int nfull = VEC ? (int)((ve - vb) / kPjVox) : 0;
  const int lrow = lane & 15, kg = lane >> 4;
  // rows past C read row C - 1 and are zeroed (no branch on the label)
  const TP* prow[4];
  bool pok[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t lab = (int64_t)lt * kPjLab + lg * 64 + t * 16 + lrow;
    pok[t] = lab < C;
    prow[t] = P + (pok[t] ? lab : (int64_t)C - 1) * N;
  }
  // a stage's tile: 16-byte pieces (column p / 8, voxels 8 (p % 8) .. +7).  A piece that starts inside the chunk
  // ends inside it (chunk ends are multiples of 64) or, in the last chunk, inside Qs's zero padding past N.
  // Threads past the tile's pieces load its last piece again and do not store it.
  uint4 qreg[PQ];
  auto load_stage = [&](int st, bool full) {
    const int64_t v0 = vb + (int64_t)st * kPjVox;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int p = min(tid + kPjThreads * q, PIECES - 1);
      const int64_t v = v0 + 8 * (p & 7);
      const bool ok = full || v < ve;
      const uint4 x = *reinterpret_cast<const uint4*>(Qs + (int64_t)(p >> 3) * Np + (ok ? v : 0));
      qreg[q] = ok ? x : uint4{0u, 0u, 0u, 0u};
    }
  };
  auto store_stage = [&](int buf) {
    uint16_t* dst = sQ + buf * KC * kPjRow;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int p = tid + kPjThreads * q;
      if (PQ * kPjThreads == PIECES || p < PIECES) *reinterpret_cast<uint4*>(dst + (p >> 3) * kPjRow + 8 * (p & 7)) = qreg[q];
    }
  };
  uint4 pa[4][2], pn[4][2];
  auto load_p = [&](uint4 (&dst)[4][2], int st, bool full) {
    const int64_t v0 = vb + (int64_t)st * kPjVox;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        if (full) {
          const uint4 x = load_p8<TP>(prow[t], v0 + 32 * ks + 8 * kg, ve, true, true);
          dst[t][ks] = pok[t] ? x : uint4{0u, 0u, 0u, 0u};
        } else {
          dst[t][ks] = load_p8<TP>(prow[t], v0 + 32 * ks + 8 * kg, ve, pok[t], VEC);
        }
      }
  };
  f4 acc[4][NH];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int c = 0; c < NH; ++c) acc[t][c] = f4{0.f, 0.f, 0.f, 0.f};
  // one stage: 2 NH column fragments from LDS, each read one step before its 4 products
  auto compute = [&](const uint4 (&pf)[4][2], int buf, bool loads_first) {
    // the next stage's global loads (issued before this call) go ahead of the products
    if (loads_first) __builtin_amdgcn_sched_group_barrier(0x020, 8 + PQ, 0);
    const uint16_t* src = sQ + buf * KC * kPjRow + (c0 * 16 + lrow) * kPjRow + 8 * kg;
    uint4 bn = *reinterpret_cast<const uint4*>(src);
#pragma unroll
    for (int q = 0; q < 2 * NH; ++q) {
      const int ks = q / NH, c = q % NH;
      const uint4 b = bn;
      if (q + 1 < 2 * NH)
        bn = *reinterpret_cast<const uint4*>(src + ((q + 1) % NH) * 16 * kPjRow + 32 * ((q + 1) / NH));
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t][c] = mfma_bf16(pf[t][ks], b, acc[t][c]);
    }
    // keep each fragment read one group of products ahead of its use (the scheduler would sink it)
    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
    for (int q = 0; q < 2 * NH - 2; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
  };
  // stage st computes from (pa, buffer st % 2) while stage st + 1's data arrive in (pn, registers)
  const bool full0 = 0 < nfull;
  load_p(pa, 0, full0);
  load_stage(0, full0);
  store_stage(0);
  __syncthreads();
  int st = 0;
  for (; st + 1 < nfull; ++st) {   // the next stage is full too: no checks
    load_p(pn, st + 1, true);
    load_stage(st + 1, true);
    compute(pa, st & 1, true);
    store_stage((st & 1) ^ 1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      pa[t][0] = pn[t][0];
      pa[t][1] = pn[t][1];
    }
    __syncthreads();
  }
  for (; st < nst; ++st) {         // the remaining stages (a partial one, or all without VEC)
    const bool more = st + 1 < nst;
    if (more) {
      const bool fn = st + 1 < nfull;
      load_p(pn, st + 1, fn);
      load_stage(st + 1, fn);
    }
    compute(pa, st & 1, false);
    if (more) {
      store_stage((st & 1) ^ 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        pa[t][0] = pn[t][0];
        pa[t][1] = pn[t][1];
      }
    }
    __syncthreads();
  }
  // D[label 4 kg + v][column lrow] of each 16 x 16 tile
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t lab = (int64_t)lt * kPjLab + lg * 64 + t * 16 + 4 * kg + v;
      if (lab >= C) continue;
      float* dst = part + (ck * C + lab) * KC + c0 * 16 + lrow;
#pragma unroll
      for (int c = 0; c < NH; ++c) dst[c * 16] = acc[t][c][v];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// projection with FP64 accumulation (FP64 and FP32 bases): a 16-column x 16-label tile per workgroup and
// voxel chunk, staged through LDS in steps of 64 voxels; the same partial layout (FP64)
// ---------------------------------------------------------------------------------------------
template <typename TQ, typename TP>
__global__ __launch_bounds__(256) void k_rwir_proj_plain(const TQ* __restrict__ Q, int ma, int64_t N,
                                                         const TP* __restrict__ P, int C,
                                                         const double* __restrict__ degree,
                                                         const double* __restrict__ sums, int normalized,
                                                         int64_t chunk, int KC, double* __restrict__ part) {
  __shared__ double sQ[16][65], sP[16][65];
  const int tid = threadIdx.x, tj = tid >> 4, tk = tid & 15;
  const int64_t ck = blockIdx.x;
  const int j0 = blockIdx.y * 16;
  const int64_t k0 = (int64_t)blockIdx.z * 16;
  const int64_t vb = ck * chunk, ve = min(N, vb + chunk);
  double acc = 0.0;
  for (int64_t v0 = vb; v0 < ve; v0 += 64) {
    // 16 rows x 64 voxels of each operand: thread (row tid / 16, voxels 4 (tid % 16) .. +3)
    const int r = tid >> 4, c4 = 4 * (tid & 15);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t v = v0 + c4 + u;
      const int j = j0 + r;
      double q = 0.0, p = 0.0;
      if (v < ve) {
        const double s = normalized ? sqrt(degree[v]) : 1.0;
        if (j < ma) q = s * (double)Elem<TQ>::ld(Q, (int64_t)j * N + v);
        else if (j == ma) q = s * ghat64(degree, sums, normalized, N, v);
        if (k0 + r < C) p = (double)Elem<TP>::ld(P, (k0 + r) * N + v);
      }
      sQ[r][c4 + u] = q;
      sP[r][c4 + u] = p;
    }
    __syncthreads();
#pragma unroll 8
    for (int u = 0; u < 64; ++u) acc = fma(sQ[tj][u], sP[tk][u], acc);
    __syncthreads();
  }
  const int j = j0 + tj;
  const int64_t k = k0 + tk;
  if (j <= ma && k < C) part[(ck * C + k) * KC + j] = acc;
}

// Z_hat(j, k) (j < ma) and g^T P_hat (j = ma): the chunk partials summed in order, FP64
template <typename TA>
__global__ void k_rwir_reduce(const TA* part, int64_t nchunk, int C, int ma, int KC, double* Zh, double* gdot) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)C * (ma + 1)) return;
  const int j = (int)(t % (ma + 1));
  const int64_t k = t / (ma + 1);
  double a = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) a += (double)part[(c * C + k) * KC + j];
  if (j < ma) Zh[j + k * ma] = a;
  else gdot[k] = a;
}

// ||p_hat_k||^2 for the sampled labels k = q step: workgroup (b, q) sums voxels b, b + kNormBlocks 256, ... of
// label k (FP64) into part[q kNormBlocks + b]; k_rwir_norms_finish adds the partials in order and puts the
// sampled labels' Z_hat columns beside them for the host: stage[q ma + j] = Z_hat(j, k), stage[ns ma + q] =
// ||p_hat_k||^2
constexpr int kNormBlocks = 64;

template <typename TP>
__global__ __launch_bounds__(256) void k_rwir_norms(const TP* P, int64_t N, int step, const double* degree,
                                                    int normalized, double* part) {
  __shared__ double sh[4];
  const int b = blockIdx.x, q = blockIdx.y, tid = threadIdx.x;
  const int64_t k = (int64_t)q * step;
  double a = 0.0;
  for (int64_t i = (int64_t)b * 256 + tid; i < N; i += (int64_t)kNormBlocks * 256) {
    const double x = (normalized ? sqrt(degree[i]) : 1.0) * (double)Elem<TP>::ld(P, k * N + i);
    a += x * x;
  }
  a = wave_sum64(a);
  if ((tid & 63) == 0) sh[tid >> 6] = a;
  __syncthreads();
  if (tid == 0) part[(int64_t)q * kNormBlocks + b] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_rwir_norms_finish(const double* part, int step, const double* Zh, int ma,
                                                           int ns, double* stage) {
  const int q = blockIdx.x, tid = threadIdx.x;
  const int64_t k = (int64_t)q * step;
  if (tid == 0) {
    double a = 0.0;
    for (int b = 0; b < kNormBlocks; ++b) a += part[(int64_t)q * kNormBlocks + b];
    stage[(int64_t)ns * ma + q] = a;
  }
  for (int j = tid; j < ma; j += 256) stage[(int64_t)q * ma + j] = Zh[j + k * ma];
}

// One wave per label: Z'(j) = g^T P_hat (j = 0) or (Z_hat(j) - c_j g^T P_hat) / n_j, Y(j) = gamma Z'(j) /
// (lambda_j + gamma), then Y(j) /= n_j (j >= 1) and kappa = sg (Y(0) - sum_{j>=1} c_j Y(j)) in Y(0) (lanes take
// j in strides, then a wave sum).  With Yt, the labels' BF16 rows for the fused reconstruction: Yt[k KR + (j -
// 1)] = Y(j) for j in [1, m), Yt[k KR + KR - 1] = kappa, zeros between; rows k in [C, Cpad) zero but for
// kPadKappa in the last column.
__global__ __launch_bounds__(256) void k_rwir_coeffs(const double* Zh, const double* gdot, int ma, int m, int C,
                                                     int Cpad, const double* lambda, double gamma, const double* cn,
                                                     const double* sums, int normalized, int64_t N, double* Y,
                                                     uint16_t* Yt, int KR) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= Cpad) return;
  if (k >= C) {
    if (Yt)
      for (int q = lane; q < KR; q += 64) Yt[k * KR + q] = q == KR - 1 ? f32_to_bf16(kPadKappa) : (uint16_t)0;
    return;
  }
  const double gd = gdot[k];
  const double* z = Zh + k * ma;
  double* y = Y + k * m;
  double part = 0.0;
  for (int j = 1 + lane; j < m; j += 64) {
    const double zp = (z[j] - cn[j] * gd) / cn[m + j];
    const double yj = gamma * zp / (lambda[j] + gamma) / cn[m + j];
    y[j] = yj;
    part += cn[j] * yj;
    if (Yt) Yt[k * KR + (j - 1)] = f32_to_bf16((float)yj);
  }
  part = wave_sum64(part);
  if (Yt)
    for (int q = m - 1 + lane; q < KR - 1; q += 64) Yt[k * KR + q] = 0;
  if (lane == 0) {
    const double kap = ghat_scaled64(sums, normalized, N) * (gamma * gd / (lambda[0] + gamma) - part);
    y[0] = kap;
    if (Yt) Yt[k * KR + KR - 1] = f32_to_bf16((float)kap);
  }
}

// ---------------------------------------------------------------------------------------------
// labels on the matrix cores (BF16 basis)
// ---------------------------------------------------------------------------------------------
// Voxel-major copy of the basis for the fused reconstruction: Qt[i KR + q] = q_{q+1}(i) for q < ma - 1,
// Qt[i KR + KR - 1] = s_i (the column that carries kappa), zeros between.  64-voxel x 32-column tiles through
// LDS (coalesced reads along voxels, 16-byte writes along columns).
__global__ __launch_bounds__(256) void k_rwir_transpose(const uint16_t* __restrict__ Q, int ma, int64_t N,
                                                        const float* __restrict__ sv, int KR,
                                                        uint16_t* __restrict__ Qt) {
  __shared__ uint16_t t[64][34];
  const int tid = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * 64;
  const int q0 = blockIdx.y * 32;
  {
    // thread: column q0 + tid / 8, voxels v0 + 8 (tid % 8) .. +7
    const int r = tid >> 3, v8 = 8 * (tid & 7);
    const int q = q0 + r;
    const int64_t i = v0 + v8;
    uint16_t x[8];
    if (q + 1 < ma && (N & 7) == 0 && i + 8 <= N) {
      const uint4 w = *reinterpret_cast<const uint4*>(Q + (int64_t)(q + 1) * N + i);
      const uint32_t a[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[2 * u] = (uint16_t)(a[u] & 0xffffu);
        x[2 * u + 1] = (uint16_t)(a[u] >> 16);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t ie = i + e;
        x[e] = ie >= N ? (uint16_t)0
                       : (q + 1 < ma ? Q[(int64_t)(q + 1) * N + ie] : (q == KR - 1 ? f32_to_bf16(sv[ie]) : (uint16_t)0));
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) t[v8 + e][r] = x[e];
  }
  __syncthreads();
  // each thread writes 8 columns (16 bytes) of one voxel: 64 voxels x 4 pieces
  const int v = tid >> 2, p = tid & 3;
  const int64_t i = v0 + v;
  if (i < N) {
    uint32_t w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = (uint32_t)t[v][8 * p + 2 * u] | ((uint32_t)t[v][8 * p + 2 * u + 1] << 16);
    *reinterpret_cast<uint4*>(Qt + i * KR + q0 + 8 * p) = uint4{w[0], w[1], w[2], w[3]};
  }
}

// Workgroup: 8 waves (two per SIMD, so that one wave's comparisons run beside the other's products) x 4
// sub-tiles of 16 voxels.  A wave keeps its 64 voxels' basis fragments (KS K steps of 32) in registers; the
// label rows go through LDS two tiles of 16 at a time (double-buffered, rows padded by 8 elements for
// conflict-free 16-byte reads, one barrier per pair), and every wave runs over all labels:
// D[label 4 kg + v][voxel lrow] = s_i U(label, i).  The larger value is kept per lane (labels in increasing
// order, strict comparison), then the four lanes of a voxel merged (larger value, or equal value and smaller
// label).  Rows of Yt past C carry -1e30 against the s column and never win.  label[i] and prob[i] =
// s_i^{-1} D; a voxel with d_i = 0 gets label 0 and probability 0.
constexpr int kLbSub = 4;
constexpr int kLbWaves = 8;
constexpr int kLbVox = kLbWaves * 16 * kLbSub;   // voxels per workgroup

template <int KS, typename TU>
__global__ __launch_bounds__(64 * kLbWaves) void k_rwir_label_mfma(const uint16_t* __restrict__ Qt, int64_t N,
                                                                   const uint16_t* __restrict__ Yt, int Cpad,
                                                                   const float* __restrict__ inv,
                                                                   int32_t* __restrict__ label,
                                                                   TU* __restrict__ prob) {
  constexpr int KR = 32 * KS;
  constexpr int ROW = KR + 8;                      // LDS row of a label (BF16 elements)
  constexpr int PIECES = 32 * KR / 8;              // 16-byte pieces of two label tiles
  __shared__ __align__(16) uint16_t sY[2][32 * ROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lrow = lane & 15, kg = lane >> 4;
  const int64_t base = (int64_t)blockIdx.x * kLbVox + wave * (16 * kLbSub);
  uint4 b[kLbSub][KS];
#pragma unroll
  for (int u = 0; u < kLbSub; ++u) {
    const int64_t i = base + 16 * u + lrow;
    const int64_t ii = i < N ? i : N - 1;
#pragma unroll
    for (int s = 0; s < KS; ++s) b[u][s] = *reinterpret_cast<const uint4*>(Qt + ii * KR + 32 * s + 8 * kg);
  }
  float best[kLbSub];
  int bidx[kLbSub];
#pragma unroll
  for (int u = 0; u < kLbSub; ++u) {
    best[u] = -INFINITY;
    bidx[u] = 0;
  }
  const int npair = Cpad >> 5;
  // a pair's rows: piece p = row p / (KR / 8), 8 elements at 8 (p % (KR / 8)), thread t takes pieces t and
  // t + 512 (at most 1024 pieces); threads past the pieces repeat the last one and do not store it
  static_assert(PIECES <= 2 * 64 * kLbWaves, "two staged pieces per thread");
  uint4 st0, st1;
  auto piece = [&](int pr, int p) {
    const int q = min(p, PIECES - 1);
    return *reinterpret_cast<const uint4*>(Yt + ((int64_t)pr * 32 + q / (KR / 8)) * KR + 8 * (q % (KR / 8)));
  };
  auto load_pair = [&](int pr) {
    st0 = piece(pr, tid);
    st1 = piece(pr, tid + 64 * kLbWaves);
  };
  auto store_pair = [&](int buf) {
    const int p0 = tid, p1 = tid + 64 * kLbWaves;
    if (p0 < PIECES) *reinterpret_cast<uint4*>(&sY[buf][(p0 / (KR / 8)) * ROW + 8 * (p0 % (KR / 8))]) = st0;
    if (p1 < PIECES) *reinterpret_cast<uint4*>(&sY[buf][(p1 / (KR / 8)) * ROW + 8 * (p1 % (KR / 8))]) = st1;
  };
  load_pair(0);
  store_pair(0);
  __syncthreads();
  for (int pr = 0; pr < npair; ++pr) {
    const int buf = pr & 1;
    if (pr + 1 < npair) load_pair(pr + 1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint4 a[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s)
        a[s] = *reinterpret_cast<const uint4*>(&sY[buf][(16 * h + lrow) * ROW + 32 * s + 8 * kg]);
      f4 c[kLbSub];
#pragma unroll
      for (int u = 0; u < kLbSub; ++u) c[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int u = 0; u < kLbSub; ++u) c[u] = mfma_bf16(a[s], b[u][s], c[u]);
      const int l0 = pr * 32 + 16 * h + 4 * kg;
#pragma unroll
      for (int u = 0; u < kLbSub; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float x = c[u][v];
          const bool gt = x > best[u];
          best[u] = gt ? x : best[u];
          bidx[u] = gt ? l0 + v : bidx[u];
        }
    }
    if (pr + 1 < npair) store_pair(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < kLbSub; ++u) {
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      const float ov = __shfl_xor(best[u], off);
      const int oi = __shfl_xor(bidx[u], off);
      if (ov > best[u] || (ov == best[u] && oi < bidx[u])) {
        best[u] = ov;
        bidx[u] = oi;
      }
    }
    const int64_t i = base + 16 * u + lrow;
    if (kg == 0 && i < N) {
      const float is = inv[i];
      label[i] = is > 0.0f ? bidx[u] : 0;
      prob[i] = (TU)(is > 0.0f ? best[u] * is : 0.0f);
    }
  }
}

// Labels with one thread per voxel (FP64 and FP32 bases): U(c, i) = s_i sum_{j>=1} q_j(i) Y(j, c) + kappa_c,
// evaluated as the reconstruction does (same operations in the same order, labels 8 at a time), the first
// label of largest U kept.
template <typename TQ, typename TU>
__global__ __launch_bounds__(256) void k_rwir_label_plain(const TQ* __restrict__ Q, int64_t N, int m,
                                                          const double* __restrict__ Y, int C,
                                                          const TU* __restrict__ dinv, int normalized,
                                                          int32_t* __restrict__ label, TU* __restrict__ prob) {
  using CT = typename Elem<TQ>::C;
  constexpr int CB = 8;
  extern __shared__ char smem[];
  CT* sY = reinterpret_cast<CT*>(smem);   // (m - 1) x CB
  CT* sK = sY + (m - 1) * CB;             // CB
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ic = i < N ? i : N - 1;
  const TQ* Q1 = Q + N;
  const int mq = m - 1;
  const CT sc = normalized ? (CT)dinv[ic] : CT(1);
  const bool live = !normalized || sc > CT(0);
  TU best = TU(0);
  int bi = -1;
  for (int lab0 = 0; lab0 < C; lab0 += CB) {
    __syncthreads();
    for (int t = threadIdx.x; t < m * CB; t += blockDim.x) {
      const int j = t / CB, c = t % CB;
      const int lab = lab0 + c;
      const CT v = lab < C ? (CT)Y[j + (int64_t)lab * m] : CT(0);
      if (j == 0) sK[c] = v;
      else sY[(j - 1) * CB + c] = v;
    }
    __syncthreads();
    CT acc[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[c] = CT(0);
    int j = 0;
    for (; j + 4 <= mq; j += 4) {
      const CT q0 = Elem<TQ>::ld(Q1, (int64_t)j * N + ic);
      const CT q1 = Elem<TQ>::ld(Q1, (int64_t)(j + 1) * N + ic);
      const CT q2 = Elem<TQ>::ld(Q1, (int64_t)(j + 2) * N + ic);
      const CT q3 = Elem<TQ>::ld(Q1, (int64_t)(j + 3) * N + ic);
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        acc[c] = fma(q0, sY[(j + 0) * CB + c], acc[c]);
        acc[c] = fma(q1, sY[(j + 1) * CB + c], acc[c]);
        acc[c] = fma(q2, sY[(j + 2) * CB + c], acc[c]);
        acc[c] = fma(q3, sY[(j + 3) * CB + c], acc[c]);
      }
    }
    for (; j < mq; ++j) {
      const CT q = Elem<TQ>::ld(Q1, (int64_t)j * N + ic);
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[c] = fma(q, sY[j * CB + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int lab = lab0 + c;
      if (lab >= C) break;
      const TU u = (TU)(sc * acc[c] + (live ? sK[c] : CT(0)));
      if (bi < 0 || u > best) {
        best = u;
        bi = lab;
      }
    }
  }
  if (i < N) {
    label[i] = live ? bi : 0;
    prob[i] = live ? best : TU(0);
  }
}

__global__ void k_rwir_zero_map(uint8_t* map, int64_t N) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) map[i] = 0;
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
constexpr int64_t kPjChunks = 64;       // voxel chunks of the matrix-core projection
constexpr int kPlainChunk = 16384;      // voxels per chunk of the FP64-accumulated projection

struct RwirDims {
  int ma, C, KC, KR, Cpad, ns, step;
  int64_t nchunk, chunk, nlt, Np;
  bool mfma;
};

static RwirDims rwir_dims(const Graph* g, int qdt, int ma, int C, int r) {
  RwirDims d;
  d.ma = ma;
  d.C = C;
  d.mfma = qdt == RW_BF16;
  // staged columns of the projection (the ma stored columns and g): the matrix-core kernel's width, else 16s
  const int nct = (ma + 1 + 15) / 16;
  d.KC = 16 * (d.mfma ? (nct <= 4 ? 4 : (nct <= 8 ? 8 : 14)) : nct);
  d.KR = (ma + 31) / 32 * 32;          // columns 1 .. ma-1, zeros, kappa's column last
  d.Cpad = (C + 31) / 32 * 32;   // label tiles of 16, taken in pairs
  d.Np = (g->N + 7) / 8 * 8;
  int step = 1;
  for (int q = 0; q < g->ndim; ++q) step *= std::max(1, r);
  d.step = step;
  d.ns = (C + step - 1) / step;
  if (d.mfma) {
    d.nchunk = std::min<int64_t>(kPjChunks, (g->N + kPjVox - 1) / kPjVox);
    d.chunk = ((g->N + d.nchunk - 1) / d.nchunk + kPjVox - 1) / kPjVox * kPjVox;
    d.nchunk = (g->N + d.chunk - 1) / d.chunk;
    d.nlt = (C + kPjLab - 1) / kPjLab;
  } else {
    d.chunk = kPlainChunk;
    d.nchunk = (g->N + d.chunk - 1) / d.chunk;
    d.nlt = 0;
  }
  return d;
}

struct RwirWork {
  float *sv, *sg, *inv;
  void* part;
  double *Zh, *gdot, *Y, *cn, *npart, *stage, *npart2;
  int* nbad;
  uint8_t* map;
  uint16_t *Yt, *Qt, *Qs;
};

static size_t rwir_layout(const Graph* g, const RwirDims& d, bool labels, void* base, RwirWork* w) {
  Carver c(base);
  RwirWork t;
  t.sv = c.take<float>(g->N);
  t.sg = c.take<float>(g->N);
  t.inv = c.take<float>(g->N);
  t.part = d.mfma ? (void*)c.take<float>((size_t)d.nchunk * d.C * d.KC)
                  : (void*)c.take<double>((size_t)d.nchunk * d.C * d.KC);
  t.Zh = c.take<double>((size_t)d.ma * d.C);
  t.gdot = c.take<double>(d.C);
  t.Y = c.take<double>((size_t)d.ma * d.C);
  t.cn = c.take<double>(2 * (size_t)d.ma);
  t.npart = c.take<double>(null_stats_partial_count(g->N, d.ma));
  t.stage = c.take<double>((size_t)d.ns * d.ma + d.ns);
  t.npart2 = c.take<double>((size_t)d.ns * kNormBlocks);
  t.nbad = c.take<int>(1);
  t.map = c.take<uint8_t>(g->N);
  t.Yt = (d.mfma && labels) ? c.take<uint16_t>((size_t)d.Cpad * d.KR) : nullptr;
  t.Qt = (d.mfma && labels) ? c.take<uint16_t>((size_t)g->N * d.KR) : nullptr;
  t.Qs = d.mfma ? c.take<uint16_t>((size_t)d.KC * d.Np) : nullptr;
  if (w) *w = t;
  return c.used + 256;
}

template <typename TP, int NH, bool VEC>
static int launch_proj(const Graph* g, const uint16_t* Q, const RwirDims& d, const void* P, const RwirWork& w,
                       hipStream_t s) {
  static bool attr = false;
  const size_t lds = rwir_proj_lds(32 * NH);
  if (!attr) {
    RW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_rwir_proj<TP, NH, VEC>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  const int64_t nwg = d.nchunk * d.nlt;
  const int64_t grid = (nwg + 7) / 8 * 8;
  k_rwir_scaled_basis<<<nblocks(d.Np / 8 * d.KC, 256), 256, 0, s>>>(Q, d.ma, g->N, d.Np, d.KC, w.sv, w.sg, w.Qs);
  RW_LAUNCH_CHECK();
  k_rwir_proj<TP, NH, VEC><<<(unsigned)grid, kPjThreads, lds, s>>>(w.Qs, d.Np, g->N, static_cast<const TP*>(P), d.C,
                                                               d.chunk, (int)d.nlt, nwg, static_cast<float*>(w.part));
  RW_LAUNCH_CHECK();
  return RW_OK;
}

template <typename TP>
static int proj_mfma(const Graph* g, const uint16_t* Q, const RwirDims& d, const void* P, const RwirWork& w,
                     hipStream_t s) {
  // d.KC is the kernel's width (the partial layout's stride)
  const bool vec = (g->N & 7) == 0;
  if (d.KC == 64) return vec ? launch_proj<TP, 2, true>(g, Q, d, P, w, s) : launch_proj<TP, 2, false>(g, Q, d, P, w, s);
  if (d.KC == 128) return vec ? launch_proj<TP, 4, true>(g, Q, d, P, w, s) : launch_proj<TP, 4, false>(g, Q, d, P, w, s);
  return vec ? launch_proj<TP, 7, true>(g, Q, d, P, w, s) : launch_proj<TP, 7, false>(g, Q, d, P, w, s);
}

template <int KS>
static int label_mfma_t(const Graph* g, const RwirDims& d, const RwirWork& w, int32_t* label, void* prob,
                        hipStream_t s) {
  const unsigned nb = (unsigned)((g->N + kLbVox - 1) / kLbVox);
  if (g->dtype == RW_F64)
    k_rwir_label_mfma<KS, double><<<nb, 64 * kLbWaves, 0, s>>>(w.Qt, g->N, w.Yt, d.Cpad, w.inv, label,
                                                               static_cast<double*>(prob));
  else
    k_rwir_label_mfma<KS, float><<<nb, 64 * kLbWaves, 0, s>>>(w.Qt, g->N, w.Yt, d.Cpad, w.inv, label,
                                                              static_cast<float*>(prob));
  RW_LAUNCH_CHECK();
  return RW_OK;
}

template <typename TQ, typename TU>
static int label_plain_t(const Graph* g, const void* Q, int m, const double* Y, int C, int32_t* label, void* prob,
                         hipStream_t s) {
  using CT = typename Elem<TQ>::C;
  const size_t sh = (size_t)m * 8 * sizeof(CT);
  k_rwir_label_plain<TQ, TU><<<nblocks(g->N, 256), 256, sh, s>>>(static_cast<const TQ*>(Q), g->N, m, Y, C,
                                                                 static_cast<const TU*>(g->dinv), g->normalized,
                                                                 label, static_cast<TU*>(prob));
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_solve_priors_workspace_bytes(rw_graph h, int q_dtype, int m_avail, int C, int r, int labels, size_t* bytes) {
  RW_CHECK(h != nullptr && bytes != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(q_dtype == RW_F64 || q_dtype == RW_F32 || q_dtype == RW_BF16, RW_EINVAL,
           "the basis is RW_F64, RW_F32 or RW_BF16");
  RW_CHECK(m_avail >= 2 && C >= 1, RW_EINVAL, "bad sizes (m_avail = %d, C = %d)", m_avail, C);
  const RwirDims d = rwir_dims(&h->g, q_dtype, m_avail, C, r);
  *bytes = rwir_layout(&h->g, d, labels != 0, nullptr, nullptr);
  return RW_OK;
}

int rw_solve_priors(rw_graph h, const void* Q, int q_dtype, const double* lambda, int m_avail, const void* prior,
                    int prior_dtype, int C, double gamma, double eps, int r, void* U, int32_t* label, void* prob,
                    void* work, size_t work_bytes, hipStream_t stream, rw_solve_info* info) {
  RW_CHECK(h != nullptr && Q != nullptr && lambda != nullptr && prior != nullptr && work != nullptr, RW_EINVAL,
           "null argument");
  RW_CHECK(q_dtype == RW_F64 || q_dtype == RW_F32 || q_dtype == RW_BF16, RW_EINVAL,
           "the basis is RW_F64, RW_F32 or RW_BF16");
  RW_CHECK(m_avail >= 2 && C >= 1, RW_EINVAL, "bad sizes (m_avail = %d, C = %d)", m_avail, C);
  RW_CHECK(gamma > 0.0, RW_EINVAL, "gamma must be > 0");
  RW_CHECK(U != nullptr || label != nullptr, RW_EINVAL, "nothing to compute: U and label are both null");
  RW_CHECK((label == nullptr) == (prob == nullptr), RW_EINVAL, "label and prob go together");
  RW_CHECK(eps <= 0.0 || r >= 1, RW_EINVAL, "r must be >= 1");
  const Graph* g = &h->g;
  const bool mf = q_dtype == RW_BF16;
  RW_CHECK(mf ? (prior_dtype == RW_BF16 || prior_dtype == RW_F32)
              : (prior_dtype == RW_F64 || prior_dtype == RW_F32),
           RW_EINVAL, "priors: RW_BF16 or RW_F32 with a BF16 basis, RW_F64 or RW_F32 otherwise");
  RW_CHECK(!mf || m_avail + 1 <= 14 * 16, RW_EINVAL, "a BF16 basis takes m_avail <= %d here (got %d)", 14 * 16 - 1,
           m_avail);
  RW_CHECK(!mf || (m_avail + 31) / 32 <= 8, RW_EINVAL, "m_avail too large for the label kernel");
  RW_CHECK((int64_t)C * g->N < ((int64_t)1 << 62), RW_EINVAL, "C x N too large");
  RW_NOT_CAPTURING(stream);
  const RwirDims d = rwir_dims(g, q_dtype, m_avail, C, r);
  RwirWork w;
  const size_t need = rwir_layout(g, d, label != nullptr, nullptr, nullptr);
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "workspace too small: %zu < %zu", work_bytes, need);
  rwir_layout(g, d, label != nullptr, work, &w);
  k_rwir_scales<<<nblocks(g->N, 256), 256, 0, stream>>>(g->degree, g->sums, g->normalized, g->N, w.sv, w.sg, w.inv);
  RW_LAUNCH_CHECK();
  // projection
  const int64_t nred = (int64_t)C * (m_avail + 1);
  if (mf) {
    const uint16_t* Qb = static_cast<const uint16_t*>(Q);
    if (prior_dtype == RW_BF16) RW_TRY(proj_mfma<uint16_t>(g, Qb, d, prior, w, stream));
    else RW_TRY(proj_mfma<float>(g, Qb, d, prior, w, stream));
    k_rwir_reduce<float><<<nblocks(nred, 256), 256, 0, stream>>>(static_cast<const float*>(w.part), d.nchunk, C,
                                                                  m_avail, d.KC, w.Zh, w.gdot);
  } else {
    const dim3 grid((unsigned)d.nchunk, (unsigned)((m_avail + 1 + 15) / 16), (unsigned)((C + 15) / 16));
    RW_CHECK(grid.z <= 65535u, RW_EINVAL, "C too large for the FP64-accumulated projection");
    double* pp = static_cast<double*>(w.part);
#define RW_PP(TQ, TP)                                                                                           \
  k_rwir_proj_plain<TQ, TP><<<grid, 256, 0, stream>>>(static_cast<const TQ*>(Q), m_avail, g->N,                 \
                                                      static_cast<const TP*>(prior), C, g->degree, g->sums,     \
                                                      g->normalized, d.chunk, d.KC, pp)
    if (q_dtype == RW_F64) {
      if (prior_dtype == RW_F64) RW_PP(double, double);
      else RW_PP(double, float);
    } else {
      if (prior_dtype == RW_F64) RW_PP(float, double);
      else RW_PP(float, float);
    }
#undef RW_PP
    RW_LAUNCH_CHECK();
    k_rwir_reduce<double><<<nblocks(nred, 256), 256, 0, stream>>>(pp, d.nchunk, C, m_avail, d.KC, w.Zh, w.gdot);
  }
  RW_LAUNCH_CHECK();
  // choice of m (eq. (25)) on the sampled labels
  int m = m_avail;
  double gmax = 0.0, gworst = 0.0;
  if (eps > 0.0) {
    const dim3 ng(kNormBlocks, (unsigned)d.ns);
    if (prior_dtype == RW_F64)
      k_rwir_norms<double><<<ng, 256, 0, stream>>>(static_cast<const double*>(prior), g->N, d.step, g->degree,
                                                   g->normalized, w.npart2);
    else if (prior_dtype == RW_F32)
      k_rwir_norms<float><<<ng, 256, 0, stream>>>(static_cast<const float*>(prior), g->N, d.step, g->degree,
                                                  g->normalized, w.npart2);
    else
      k_rwir_norms<uint16_t><<<ng, 256, 0, stream>>>(static_cast<const uint16_t*>(prior), g->N, d.step, g->degree,
                                                     g->normalized, w.npart2);
    RW_LAUNCH_CHECK();
    k_rwir_norms_finish<<<d.ns, 256, 0, stream>>>(w.npart2, d.step, w.Zh, m_avail, d.ns, w.stage);
    RW_LAUNCH_CHECK();
    const size_t nst = (size_t)d.ns * m_avail + d.ns;
    void* stage = nullptr;
    RW_TRY(host_stage((nst + 1) * sizeof(double), &stage));
    double* hz = static_cast<double*>(stage);
    RW_HIP(hipMemcpyAsync(hz, w.stage, nst * sizeof(double), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipMemcpyAsync(hz + nst, g->sums, sizeof(double), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipStreamSynchronize(stream));
    gmax = eps * eps * (g->normalized ? hz[nst] : (double)g->N);
    std::vector<double> gk(hz + (size_t)d.ns * m_avail, hz + nst);
    for (int mm = 1; mm <= m_avail; ++mm) {
      double worst = 0.0;
      for (int q = 0; q < d.ns; ++q) {
        const double z = hz[(size_t)q * m_avail + (mm - 1)];
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
  // the FP64 basis of the first m columns and the coefficients
  RW_TRY(fill_i32(w.nbad, 1, 0, stream));
  RW_TRY(null_stats(g, Q, q_dtype, m, w.npart, w.cn, w.nbad, stream));
  const bool fused = mf && label != nullptr;
  k_rwir_coeffs<<<nblocks(d.Cpad, 4), 256, 0, stream>>>(w.Zh, w.gdot, m_avail, m, C, d.Cpad, lambda, gamma, w.cn,
                                                          g->sums, g->normalized, g->N, w.Y,
                                                          fused ? w.Yt : nullptr, d.KR);
  RW_LAUNCH_CHECK();
  if (U != nullptr) {
    k_rwir_zero_map<<<nblocks(g->N, 256), 256, 0, stream>>>(w.map, g->N);
    RW_LAUNCH_CHECK();
    RW_TRY(reconstruct_any(g, Q, q_dtype, m, w.Y, C, w.map, U, stream));
  }
  if (label != nullptr) {
    if (fused) {
      const dim3 tg((unsigned)((g->N + 63) / 64), (unsigned)(d.KR / 32));
      k_rwir_transpose<<<tg, 256, 0, stream>>>(static_cast<const uint16_t*>(Q), m, g->N, w.sv, d.KR, w.Qt);
      RW_LAUNCH_CHECK();
      switch (d.KR / 32) {
        case 1: RW_TRY(label_mfma_t<1>(g, d, w, label, prob, stream)); break;
        case 2: RW_TRY(label_mfma_t<2>(g, d, w, label, prob, stream)); break;
        case 3: RW_TRY(label_mfma_t<3>(g, d, w, label, prob, stream)); break;
        case 4: RW_TRY(label_mfma_t<4>(g, d, w, label, prob, stream)); break;
        case 5: RW_TRY(label_mfma_t<5>(g, d, w, label, prob, stream)); break;
        case 6: RW_TRY(label_mfma_t<6>(g, d, w, label, prob, stream)); break;
        case 7: RW_TRY(label_mfma_t<7>(g, d, w, label, prob, stream)); break;
        default: RW_TRY(label_mfma_t<8>(g, d, w, label, prob, stream)); break;
      }
    } else {
      RW_CHECK((size_t)m * 8 * 8 <= 65536, RW_EINVAL, "m = %d too large for the label kernel", m);
      if (g->dtype == RW_F64) {
        if (q_dtype == RW_F64) RW_TRY((label_plain_t<double, double>(g, Q, m, w.Y, C, label, prob, stream)));
        else RW_TRY((label_plain_t<float, double>(g, Q, m, w.Y, C, label, prob, stream)));
      } else {
        if (q_dtype == RW_F64) RW_TRY((label_plain_t<double, float>(g, Q, m, w.Y, C, label, prob, stream)));
        else RW_TRY((label_plain_t<float, float>(g, Q, m, w.Y, C, label, prob, stream)));
      }
    }
  }
  void* stage = nullptr;
  RW_TRY(host_stage(sizeof(int), &stage));
  RW_HIP(hipMemcpyAsync(stage, w.nbad, sizeof(int), hipMemcpyDeviceToHost, stream));
  RW_HIP(hipStreamSynchronize(stream));
  int nbad = 0;
  std::memcpy(&nbad, stage, sizeof(int));
  RW_CHECK(!nbad, RW_EINVAL, "basis column %d lies in the span of the null vector (column 0)", nbad);
  if (info) {
    info->m_used = m;
    info->eig_probes = 0;
    info->f_max = gmax;
    info->f_worst = gworst;
    info->min_pivot = 1.0;
  }
  return RW_OK;
}

}  // extern "C"
