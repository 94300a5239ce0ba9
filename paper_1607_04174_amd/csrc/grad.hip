// Gradients of a loss on the random-walker probabilities through the exact (gamma = 0) solution of
// Sec. II-A eq. (5): with L = sum_e w_e (e_i - e_j)(e_i - e_j)^T and the adjoint A = L_n^{-1} G
// (zero on seeds) of the loss gradient G = dl/dU, differentiating L_n U_n = -B^T U_s gives
//   dl/dw_e = -sum_k (a_i^k - a_j^k)(u_i^k - u_j^k),
// and the chain through w_e = s_e exp(-beta f(J_i - J_j)) of eq. (2) gives the gradients for the
// intensities, beta and the per-edge scales.  Also: per-edge scale input, and the spectral
// approximation of the pseudo-inverse used as the adjoint solve's starting point.
#include <cmath>

#include "rw_internal.h"

namespace rw {

// per node i and forward direction d: dl/dw, dl/ds and the beta partial sums
__global__ void k_grad_edges(GridDev G, int form, double beta, const double* J, const double* weight,
                             const uint8_t* mask, const double* U, const double* A, int C, double* dw, double* ds,
                             double* partial) {
  double local = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G.N; i += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t m = mask[i];
    for (int d = 0; d < G.ndir; ++d) {
      double g = 0.0, gs = 0.0;
      if ((m >> d) & 1u) {
        const int64_t j = i + G.off[d];
        for (int k = 0; k < C; ++k) {
          const int64_t o = (int64_t)k * G.N;
          g -= (A[o + i] - A[o + j]) * (U[o + i] - U[o + j]);
        }
        const double diff = J[i] - J[j];
        const double f = form == RW_WEIGHT_SQUARED ? diff * diff : fabs(diff);
        gs = g * exp(-beta * f);
        local += g * weight[d * G.N + i] * (-f);
      }
      dw[d * G.N + i] = g;
      ds[d * G.N + i] = gs;
    }
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = local;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_grad_sum(const double* partial, int n, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    out[0] = s;
  }
}

// dl/dJ_i: node i is the tail of its forward edges and the head of the backward ones
__global__ void k_grad_J(GridDev G, int form, double beta, const double* J, const double* weight, const uint8_t* mask,
                         const double* dw, double* dJ) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  const int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / (G.nx * G.ny);
  double acc = 0.0;
  const uint8_t m = mask[i];
  for (int d = 0; d < G.ndir; ++d) {
    if ((m >> d) & 1u) {   // edge (i, j): dw/dJ_i = w * (-beta f'(J_i - J_j))
      const double diff = J[i] - J[i + G.off[d]];
      const double fp = form == RW_WEIGHT_SQUARED ? 2.0 * diff : (diff > 0.0 ? 1.0 : (diff < 0.0 ? -1.0 : 0.0));
      acc += dw[d * G.N + i] * weight[d * G.N + i] * (-beta * fp);
    }
    if (tail_in(G, x, y, z, d)) {
      const int64_t t = i - G.off[d];
      if ((mask[t] >> d) & 1u) {   // edge (t, i): dw/dJ_i = w * (+beta f'(J_t - J_i))
        const double diff = J[t] - J[i];
        const double fp = form == RW_WEIGHT_SQUARED ? 2.0 * diff : (diff > 0.0 ? 1.0 : (diff < 0.0 ? -1.0 : 0.0));
        acc += dw[d * G.N + t] * weight[d * G.N + t] * (beta * fp);
      }
    }
  }
  dJ[i] = acc;
}

__global__ void k_set_scale(GridDev G, const double* in, const uint8_t* mask, double* scale) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  const uint8_t m = mask[i];
  for (int d = 0; d < G.ndir; ++d) scale[d * G.N + i] = ((m >> d) & 1u) ? in[d * G.N + i] : 0.0;
}

// Y(k, i) = s_i B(k, i) with s = d^{-1/2} (normalized) or 1
__global__ void k_scale_rows(const double* B, const double* dinv, int normalized, int64_t N, int C, double* Y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= N) return;
  Y[(int64_t)k * N + i] = normalized ? dinv[i] * B[(int64_t)k * N + i] : B[(int64_t)k * N + i];
}

// T(j, k) /= lambda_j for j >= 1, T(0, k) = 0 (the null pair is left out)
__global__ void k_div_lambda(double* T, const double* lambda, int m, int C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * C) return;
  const int j = t % m;
  T[t] = (j == 0 || lambda[j] == 0.0) ? 0.0 : T[t] / lambda[j];
}

static size_t spectral_layout(const Graph* g, int m, int C, void* base, double** Y, double** T, double** partial) {
  Carver c(base);
  double* y = c.take<double>((size_t)C * g->N);
  double* t = c.take<double>((size_t)m * C);
  double* p = c.take<double>(gram_partial_count(g->N, m, C));
  if (Y) { *Y = y; *T = t; *partial = p; }
  return c.used;
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_graph_set_scale(rw_graph h, const void* scale, hipStream_t stream) {
  RW_CHECK(h != nullptr && scale != nullptr, RW_EINVAL, "null argument");
  Graph* g = &h->g;
  GridDev G = grid_of(g);
  k_set_scale<<<nblocks(g->N, 256), 256, 0, stream>>>(G, (const double*)scale, g->mask, g->scale);
  RW_LAUNCH_CHECK();
  return graph_rebuild(g, stream);
}

int rw_grad_workspace_bytes(rw_graph h, size_t* bytes) {
  RW_CHECK(h != nullptr && bytes != nullptr, RW_EINVAL, "null argument");
  *bytes = kReduceBlocks * sizeof(double);
  return RW_OK;
}

int rw_grad_edges(rw_graph h, const double* U, const double* A, int C, double* dw, double* dJ, double* dbeta,
                  double* ds, void* work, size_t work_bytes, hipStream_t stream) {
  RW_CHECK(h != nullptr && U != nullptr && A != nullptr && dw != nullptr && dJ != nullptr && dbeta != nullptr &&
               ds != nullptr && work != nullptr, RW_EINVAL, "null argument");
  const Graph* g = &h->g;
  RW_CHECK(g->dtype == RW_F64, RW_EINVAL, "gradients need an FP64 graph");
  RW_CHECK(C >= 1, RW_EINVAL, "C must be >= 1");
  RW_CHECK(work_bytes >= kReduceBlocks * sizeof(double), RW_EWORKSPACE, "gradient workspace too small");
  GridDev G = grid_of(g);
  double* partial = static_cast<double*>(work);
  const int nb = (int)std::min<int64_t>(kReduceBlocks, nblocks(g->N, 256));
  k_grad_edges<<<nb, 256, 0, stream>>>(G, g->weight_form, g->beta, g->J, (const double*)g->weight, g->mask, U, A, C, dw,
                                        ds, partial);
  RW_LAUNCH_CHECK();
  k_grad_sum<<<1, 64, 0, stream>>>(partial, nb, dbeta);
  k_grad_J<<<nblocks(g->N, 256), 256, 0, stream>>>(G, g->weight_form, g->beta, g->J, (const double*)g->weight, g->mask,
                                                   dw, dJ);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

int rw_spectral_workspace_bytes(rw_graph h, int m, int C, size_t* bytes) {
  RW_CHECK(h != nullptr && bytes != nullptr && m >= 1 && C >= 1, RW_EINVAL, "bad argument");
  *bytes = spectral_layout(&h->g, m, C, nullptr, nullptr, nullptr, nullptr);
  return RW_OK;
}

int rw_spectral_apply(rw_graph h, const double* Q, const double* lambda, int m, const double* B, int C, double* X,
                      void* work, size_t work_bytes, hipStream_t stream) {
  RW_CHECK(h != nullptr && Q != nullptr && lambda != nullptr && B != nullptr && X != nullptr && work != nullptr,
           RW_EINVAL, "null argument");
  const Graph* g = &h->g;
  RW_CHECK(g->dtype == RW_F64, RW_EINVAL, "the spectral approximation needs an FP64 graph");
  RW_CHECK(m >= 1 && C >= 1, RW_EINVAL, "bad sizes");
  double *Y = nullptr, *T = nullptr, *partial = nullptr;
  size_t need = spectral_layout(g, m, C, work, &Y, &T, &partial);
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "spectral workspace too small: %zu < %zu", work_bytes, need);
  dim3 gridN(nblocks(g->N, 256), C);
  k_scale_rows<<<gridN, 256, 0, stream>>>(B, (const double*)g->dinv, g->normalized, g->N, C, Y);
  RW_LAUNCH_CHECK();
  RW_TRY(gram(RW_F64, Q, g->N, Y, g->N, g->N, m, C, T, partial, stream));            // T = Q^T S B
  k_div_lambda<<<nblocks(m * C, 256), 256, 0, stream>>>(T, lambda, m, C);
  RW_LAUNCH_CHECK();
  RW_TRY(gemm_tn(RW_F64, Q, g->N, T, m, Y, g->N, g->N, m, C, 0.0, stream));          // Y = Q Lambda'^+ T
  k_scale_rows<<<gridN, 256, 0, stream>>>(Y, (const double*)g->dinv, g->normalized, g->N, C, X);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // extern "C"
