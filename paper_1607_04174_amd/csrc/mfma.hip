// BF16 tall-skinny contractions with the eigenbasis on the matrix cores (v_mfma_f32_16x16x16bf16),
// FP32 accumulation:
//   reconstruction  U = s * (Q Y)   (N x m times m x C; Sec. II-B eq. (16): the labels are linear
//                                     combinations of the eigenvectors), seed rows one-hot;
//   projection      P = Q^T X       (m x N times N x C).
// Q is stored in BF16 (half the HBM bytes of FP32); the small operand (Y or X) is split into a
// high and a low BF16 part that occupy separate MFMA output columns, so it keeps ~16 significant
// bits and the only BF16 rounding that matters is Q's.  With C <= 8 labels the 16 output columns
// hold both parts; the contraction stays HBM-bound (it reads Q once), so the matrix cores are
// lightly used by construction.
//
// MFMA 16x16x16 operand layout (wave64): lane l holds A[l % 16][4 (l / 16) + v] and
// B[4 (l / 16) + v][l % 16] for v = 0..3, and receives D[4 (l / 16) + v][l % 16].
#include "rw_internal.h"

namespace rw {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaNodes = 256;   // nodes per workgroup tile (4 waves x 64)
constexpr int kSQ = 20;           // padded row of the staged Q tile (16 k values + 4)

__device__ __forceinline__ void split_bf16(float v, uint16_t* hi, uint16_t* lo) {
  *hi = f32_to_bf16(v);
  *lo = f32_to_bf16(v - bf16_to_f32(*hi));
}

// ---------------------------------------------------------------------------------------------
// reconstruction
// ---------------------------------------------------------------------------------------------
template <typename TU>
__global__ __launch_bounds__(256) void k_reconstruct_mfma(const uint16_t* __restrict__ Q,
                                                           const uint16_t* __restrict__ Qlo, int pm, int64_t N,
                                                           int m, const double* __restrict__ Y, int C,
                                                           const uint8_t* __restrict__ map,
                                                           const TU* __restrict__ dinv, int normalized,
                                                           TU* __restrict__ U) {
  extern __shared__ char smem[];
  // the product runs over Q's columns 1 .. m-1 against Y's rows 1 .. m-1; Y's row 0 is the null vector's
  // per-label term, added in the epilogue.  With the pair form's remainder columns (Qlo, pm of them) the
  // contraction runs on over them, against Y's rows 1 .. pm again: k in [m-1, m-1+pm) reads Qlo column
  // k - (m-1).
  Q += N;
  Y += 1;
  const int ldy = m;
  m -= 1;
  const int kext = m + pm;
  const int mpad = (kext + 15) & ~15;
  uint16_t* sBt = reinterpret_cast<uint16_t*>(smem);                    // [16 cols][mpad]
  uint16_t* sQ = sBt + 16 * mpad;                                       // [256 nodes][kSQ]
  float* sD = reinterpret_cast<float*>(sQ + kMfmaNodes * kSQ);           // [256 nodes][17]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t node0 = (int64_t)blockIdx.x * kMfmaNodes;
  // B operand: columns 0..C-1 high parts, C..2C-1 low parts, zero elsewhere
  for (int t = tid; t < 16 * mpad; t += 256) {
    int col = t / mpad, k = t - col * mpad;
    uint16_t v = 0;
    if (k < kext) {
      int c = col < C ? col : col - C;
      if (col < 2 * C) {
        uint16_t hi, lo;
        split_bf16((float)Y[(k < m ? k : k - m) + (int64_t)c * ldy], &hi, &lo);
        v = col < C ? hi : lo;
      }
    }
    sBt[t] = v;
  }
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool vec = (N & 3) == 0;
  // Q[k0 .. k0+16) x [node0, node0 + 256): thread (g, kq) reads rows k0 + 4 kq .. +3 at nodes
  // node0 + 4 g .. +3 (four 8-byte loads, one step ahead of use), transposes the 4 x 4 block in
  // registers and stores each node's four k values as one 8-byte word: sQ[node][k] with a padded row
  // of kSQ elements (no bank conflicts between the 16 node rows a wave touches)
  const int kq = tid & 3, g = tid >> 2;
  const int64_t gnode = node0 + 4 * g;
  uint2 pre[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = k0 + 4 * kq + r;
      uint2 w = make_uint2(0u, 0u);
      if (k < kext) {
        const uint16_t* src = (k < m ? Q + (int64_t)k * N : Qlo + (int64_t)(k - m) * N) + gnode;
        if (vec && gnode + 3 < N) {
          w = *reinterpret_cast<const uint2*>(src);
        } else {
          const uint32_t v0 = gnode < N ? src[0] : 0u, v1 = gnode + 1 < N ? src[1] : 0u;
          const uint32_t v2 = gnode + 2 < N ? src[2] : 0u, v3 = gnode + 3 < N ? src[3] : 0u;
          w = make_uint2(v0 | (v1 << 16), v2 | (v3 << 16));
        }
      }
      pre[r] = w;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < mpad; k0 += 16) {
    __syncthreads();
    {
      const uint32_t a0 = pre[0].x, a1 = pre[1].x, a2 = pre[2].x, a3 = pre[3].x;   // nodes 0, 1
      const uint32_t b0 = pre[0].y, b1 = pre[1].y, b2 = pre[2].y, b3 = pre[3].y;   // nodes 2, 3
      uint2* dst = reinterpret_cast<uint2*>(sQ + (4 * g) * kSQ + 4 * kq);
      dst[0] = make_uint2((a0 & 0xffffu) | (a1 << 16), (a2 & 0xffffu) | (a3 << 16));
      dst[kSQ / 4] = make_uint2((a0 >> 16) | (a1 & 0xffff0000u), (a2 >> 16) | (a3 & 0xffff0000u));
      dst[2 * (kSQ / 4)] = make_uint2((b0 & 0xffffu) | (b1 << 16), (b2 & 0xffffu) | (b3 << 16));
      dst[3 * (kSQ / 4)] = make_uint2((b0 >> 16) | (b1 & 0xffff0000u), (b2 >> 16) | (b3 & 0xffff0000u));
    }
    __syncthreads();
    if (k0 + 16 < mpad) fetch(k0 + 16);
    const bf16x4 b = *reinterpret_cast<const bf16x4*>(sBt + (lane & 15) * mpad + k0 + 4 * (lane >> 4));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int nl = 64 * wave + 16 * t + (lane & 15);
      const bf16x4 a = *reinterpret_cast<const bf16x4*>(sQ + nl * kSQ + 4 * (lane >> 4));
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
  // epilogue: combine high + low columns per node through LDS
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int nl = 64 * wave + 16 * t + 4 * (lane >> 4) + v;
      sD[nl * 17 + (lane & 15)] = acc[t][v];
    }
  __syncthreads();
  const int64_t i = node0 + tid;
  if (i >= N) return;
  const int ml = map[i];
  const float sc = normalized ? (float)dinv[i] : 1.0f;
  const bool live = !normalized || sc > 0.0f;
  for (int c = 0; c < C; ++c) {
    const float val = sD[tid * 17 + c] + sD[tid * 17 + c + C];
    const float kap = live ? (float)Y[(int64_t)c * ldy - 1] : 0.0f;
    U[(int64_t)c * N + i] = ml ? (ml - 1 == c ? TU(1) : TU(0)) : TU(sc * val + kap);
  }
}

size_t reconstruct_mfma_lds(int m, int pm) {
  const int mpad = (m - 1 + pm + 15) & ~15;   // columns 1 .. m-1, then pm remainder columns
  return (size_t)16 * mpad * 2 + (size_t)kMfmaNodes * kSQ * 2 + (size_t)kMfmaNodes * 17 * 4;
}

int reconstruct_mfma(const Graph* g, const void* Q, const uint16_t* Qlo, int m, const double* Y, int C,
                     const uint8_t* map, void* U, hipStream_t s) {
  RW_CHECK(C <= 8, RW_EINVAL, "the BF16 matrix-core reconstruction handles at most 8 labels");
  const int pm = Qlo != nullptr ? std::min(kPairCols, m - 1) : 0;
  const size_t sh = reconstruct_mfma_lds(m, pm);
  RW_CHECK(sh <= 64 * 1024, RW_EINVAL, "m = %d too large for the matrix-core reconstruction tile", m);
  const unsigned grid = (unsigned)((g->N + kMfmaNodes - 1) / kMfmaNodes);
  if (g->dtype == RW_F64)
    k_reconstruct_mfma<double><<<grid, 256, sh, s>>>((const uint16_t*)Q, Qlo, pm, g->N, m, Y, C, map,
                                                     (const double*)g->dinv, g->normalized, (double*)U);
  else
    k_reconstruct_mfma<float><<<grid, 256, sh, s>>>((const uint16_t*)Q, Qlo, pm, g->N, m, Y, C, map,
                                                    (const float*)g->dinv, g->normalized, (float*)U);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

// ---------------------------------------------------------------------------------------------
// projection P = Q^T X: each workgroup accumulates a partial over its node range for every 16-row
// chunk of Q^T, then the partials are summed in FP64 in a fixed order
// ---------------------------------------------------------------------------------------------
constexpr int kProjMaxChunks = 16;   // m <= 256

__global__ __launch_bounds__(256) void k_project_mfma(const uint16_t* __restrict__ Q, int64_t N, int m,
                                                      const float* __restrict__ X, int C, int64_t nodes_per_block,
                                                      float* __restrict__ partial) {
  __shared__ float sR[4][16 * 16];           // per-wave results of one m-chunk
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool vec = (N & 3) == 0;
  const int mchunks = (m + 15) >> 4;
  const int64_t begin = (int64_t)blockIdx.x * nodes_per_block;
  const int64_t end = std::min<int64_t>(N, begin + nodes_per_block);
  f32x4 acc[kProjMaxChunks];
#pragma unroll
  for (int q = 0; q < kProjMaxChunks; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t n0 = begin; n0 < end; n0 += kMfmaNodes) {
    // B fragments (X split) for this wave's 64 nodes: 4 k-steps of 16 nodes
    bf16x4 b[4];
    const int j = lane & 15;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t nb = n0 + 64 * wave + 16 * st + 4 * (lane >> 4);
      short e[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t node = nb + v;
        uint16_t hv = 0;
        if (node < end && j < 2 * C) {
          uint16_t hi, lo;
          split_bf16(X[(int64_t)(j < C ? j : j - C) * N + node], &hi, &lo);
          hv = j < C ? hi : lo;
        }
        e[v] = (short)hv;
      }
      b[st] = bf16x4{e[0], e[1], e[2], e[3]};
    }
    // A fragments straight from HBM: lane l takes four consecutive nodes of eigenvector 16 q + (l mod 16)
    // (one 8-byte load when N is a multiple of 4), so Q needs no staging through LDS
#pragma unroll
    for (int q = 0; q < kProjMaxChunks; ++q) {
      if (q >= mchunks) break;
      const int k = 16 * q + (lane & 15);
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int64_t nb = n0 + 64 * wave + 16 * st + 4 * (lane >> 4);
        bf16x4 a = bf16x4{0, 0, 0, 0};
        if (k < m) {
          const uint16_t* src = Q + (int64_t)k * N + nb;
          if (vec && nb + 3 < end) {
            a = *reinterpret_cast<const bf16x4*>(src);
          } else {
            short e[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) e[v] = nb + v < end ? (short)src[v] : (short)0;
            a = bf16x4{e[0], e[1], e[2], e[3]};
          }
        }
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[st], acc[q], 0, 0, 0);
      }
    }
  }
  // reduce the 4 waves and write this block's partial [m][16]
  float* out = partial + (int64_t)blockIdx.x * mchunks * 256;
#pragma unroll
  for (int q = 0; q < kProjMaxChunks; ++q) {
    if (q >= mchunks) break;
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) sR[wave][(4 * (lane >> 4) + v) * 16 + (lane & 15)] = acc[q][v];
    __syncthreads();
    out[q * 256 + tid] = sR[0][tid] + sR[1][tid] + sR[2][tid] + sR[3][tid];
  }
}

// P(i, c) (leading dimension ldp) = the sum of the block partials of row i, label c (both BF16 parts of X)
__global__ void k_project_final(const float* partial, int nblocks, int m, int C, double* P, int ldp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * C) return;
  const int i = t % m, c = t / m;
  const int mchunks = (m + 15) >> 4;
  const int q = i >> 4, r = i & 15;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) {
    const float* p = partial + (int64_t)b * mchunks * 256 + q * 256 + r * 16;
    s += (double)p[c] + (double)p[c + C];
  }
  P[i + (int64_t)c * ldp] = s;
}

__global__ void k_add_rows(const double* T, int rows, int C, double* P, int ldp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * C) return;
  const int i = t % rows, c = t / rows;
  P[i + (int64_t)c * ldp] += T[t];
}

static int proj_blocks(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (N + 1023) / 1024)); }

size_t project_partial_count(int64_t N, int m) {
  return (size_t)proj_blocks(N) * ((m + 15) / 16) * 256;
}

// BF16 Q^T X on the matrix cores in blocks of at most 256 columns and 8 labels
static int project_bf16(const uint16_t* Q, int64_t N, int m, const float* X, int C, double* P, int ldp,
                        float* partial, hipStream_t s) {
  const int nb = proj_blocks(N);
  const int64_t per = ((N + nb - 1) / nb + kMfmaNodes - 1) / kMfmaNodes * kMfmaNodes;
  for (int c0 = 0; c0 < m; c0 += 16 * kProjMaxChunks)
    for (int l0 = 0; l0 < C; l0 += 8) {
      const int mc = std::min(16 * kProjMaxChunks, m - c0), cc = std::min(8, C - l0);
      k_project_mfma<<<nb, 256, 0, s>>>(Q + (int64_t)c0 * N, N, mc, X + (int64_t)l0 * N, cc, per, partial);
      RW_LAUNCH_CHECK();
      k_project_final<<<nblocks((int64_t)mc * cc, 256), 256, 0, s>>>(partial, nb, mc, cc,
                                                                       P + c0 + (int64_t)l0 * ldp, ldp);
      RW_LAUNCH_CHECK();
    }
  return RW_OK;
}

size_t project_block_partial_bytes(int64_t N, int m, int C) {
  return std::max(project_partial_count(N, std::min(m, 16 * kProjMaxChunks)) * sizeof(float),
                  project_cols_partial_count(N, m, C) * sizeof(double));
}

int project_block(const void* Q, int qdt, int64_t N, int m, const void* X, int C, double* P, void* partial,
                  double* tmp, hipStream_t s) {
  if (qdt == RW_F64 || qdt == RW_F32) return project_cols(qdt, Q, N, m, X, C, P, static_cast<double*>(partial), s);
  const BasisView b = basis_view(N, Q, qdt);
  RW_TRY(project_bf16(static_cast<const uint16_t*>(b.hi), N, m, static_cast<const float*>(X), C, P, m,
                      static_cast<float*>(partial), s));
  if (b.lo != nullptr && m > 1) {   // the remainder columns add to rows 1 .. pm
    const int pm = std::min(kPairCols, m - 1);
    RW_TRY(project_bf16(b.lo, N, pm, static_cast<const float*>(X), C, tmp, pm, static_cast<float*>(partial), s));
    k_add_rows<<<nblocks((int64_t)pm * C, 256), 256, 0, s>>>(tmp, pm, C, P + 1, m);
    RW_LAUNCH_CHECK();
  }
  return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_convert_block(const void* src, int src_dtype, void* dst, int dst_dtype, int64_t rows, int cols,
                     hipStream_t stream) {
  RW_CHECK(src != nullptr && dst != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(src != dst, RW_EINVAL, "source and destination must differ");
  RW_CHECK(rows >= 0 && cols >= 0, RW_EINVAL, "bad sizes");
  if (dst_dtype == RW_BF16_PAIR) {
    RW_CHECK(src_dtype == RW_F64 || src_dtype == RW_F32, RW_EINVAL, "the pair form is made from an F64 or F32 block");
    return convert_pair(src_dtype, src, rows, static_cast<uint16_t*>(dst), cols, stream);
  }
  RW_CHECK((src_dtype == RW_F64 || src_dtype == RW_F32 || src_dtype == RW_BF16) &&
               (dst_dtype == RW_F64 || dst_dtype == RW_F32 || dst_dtype == RW_BF16), RW_EINVAL, "bad dtype");
  return convert_block(src_dtype, src, rows, dst_dtype, dst, rows, rows, cols, stream);
}

int rw_project_workspace_bytes(int64_t N, int m, int C, size_t* bytes) {
  RW_CHECK(bytes != nullptr && N >= 1 && m >= 1 && C >= 1, RW_EINVAL, "bad sizes");
  *bytes = std::max(project_partial_count(N, m) * sizeof(float), project_cols_partial_count(N, m, C) * sizeof(double));
  return RW_OK;
}

int rw_project_basis(const void* Q, int q_dtype, int64_t N, int m, const float* X, int C, double* P, void* work,
                     size_t work_bytes, hipStream_t stream) {
  RW_CHECK(Q != nullptr && X != nullptr && P != nullptr && work != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(N >= 1 && m >= 1 && C >= 1, RW_EINVAL, "bad sizes");
  size_t need = 0;
  RW_TRY(rw_project_workspace_bytes(N, m, C, &need));
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "projection workspace too small: %zu < %zu", work_bytes, need);
  if (q_dtype == RW_F32) return project_cols(RW_F32, Q, N, m, X, C, P, static_cast<double*>(work), stream);
  RW_CHECK(q_dtype == RW_BF16, RW_EINVAL,
           "projection supports F32 (VALU) and BF16 (matrix cores) bases (a pair form's plain block is BF16)");
  RW_CHECK(C <= 8 && m <= 16 * kProjMaxChunks, RW_EINVAL, "matrix-core projection needs C <= 8 and m <= 256");
  const int nb = proj_blocks(N);
  const int64_t per = ((N + nb - 1) / nb + kMfmaNodes - 1) / kMfmaNodes * kMfmaNodes;
  float* partial = static_cast<float*>(work);
  k_project_mfma<<<nb, 256, 0, stream>>>((const uint16_t*)Q, N, m, X, C, per, partial);
  RW_LAUNCH_CHECK();
  k_project_final<<<nblocks((int64_t)m * C, 256), 256, 0, stream>>>(partial, nb, m, C, P, m);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // extern "C"
