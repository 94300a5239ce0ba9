// Prior probabilities from the seeds (Sec. IV-A): a Gaussian fitted to the intensities of each label's seeds;
// the prior of label k at voxel i is that Gaussian's density at J_i, normalized over the labels.
//   fit:    mean and maximum-likelihood variance of J over label k's seeds (FP64, two passes, fixed order),
//           variance floored at 1e-6; a label without seeds is absent (prior 0, not in the normalization)
//   prior:  softmax over the present labels of log N(J_i; mu_k, var_k) (the normalized density without
//           the underflow of exp far from every mean)
#include <cmath>

#include "rw_internal.h"

namespace rw {

constexpr double kPriorVarFloor = 1e-6;
constexpr int kFitThreads = 1024;

// one workgroup: fit[k] = mean, fit[C + k] = variance, fit[2C + k] = seed count (as a double); *status is
// RW_OK, or RW_EINVAL when a seed is out of range or carries a label outside [0, C) (such seeds are skipped)
__global__ __launch_bounds__(kFitThreads) void k_prior_fit(const double* J, int64_t N, const int64_t* node,
                                                           const int32_t* label, int64_t S, int C, double* fit,
                                                           int32_t* status) {
  __shared__ double sh[kFitThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto block_sum = [&](double v) {
    v = wave_sum64(v);
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kFitThreads / 64; ++w) t += sh[w];
    return t;
  };
  if (tid == 0) *status = RW_OK;
  __syncthreads();
  for (int64_t q = tid; q < S; q += kFitThreads)
    if (node[q] < 0 || node[q] >= N || label[q] < 0 || label[q] >= C) *status = RW_EINVAL;
  for (int k = 0; k < C; ++k) {
    double n = 0.0, s = 0.0;
    for (int64_t q = tid; q < S; q += kFitThreads) {
      const int64_t v = node[q];
      if (label[q] == k && v >= 0 && v < N) {
        n += 1.0;
        s += J[v];
      }
    }
    n = block_sum(n);
    s = block_sum(s);
    const double mu = n > 0.0 ? s / n : 0.0;
    double s2 = 0.0;
    for (int64_t q = tid; q < S; q += kFitThreads) {
      const int64_t v = node[q];
      if (label[q] == k && v >= 0 && v < N) {
        const double d = J[v] - mu;
        s2 += d * d;
      }
    }
    s2 = block_sum(s2);
    if (tid == 0) {
      fit[k] = mu;
      fit[C + k] = n > 0.0 ? fmax(s2 / n, kPriorVarFloor) : kPriorVarFloor;
      fit[2 * C + k] = n;
    }
  }
}

// one thread per voxel: two passes over the labels (the largest log-density, then the normalized terms)
template <typename TP>
__global__ __launch_bounds__(256) void k_prior_gauss(const double* J, int64_t N, int C, const double* fit,
                                                     TP* prior) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double x = J[i];
  auto logd = [&](int k) {
    const double d = x - fit[k], v = fit[C + k];
    return -0.5 * d * d / v - 0.5 * log(2.0 * M_PI * v);
  };
  double top = -INFINITY;
  for (int k = 0; k < C; ++k)
    if (fit[2 * C + k] > 0.0) top = fmax(top, logd(k));
  double sum = 0.0;
  for (int k = 0; k < C; ++k)
    if (fit[2 * C + k] > 0.0) sum += exp(logd(k) - top);
  for (int k = 0; k < C; ++k)   // no present label (every seed invalid): zeros
    prior[(int64_t)k * N + i] = (fit[2 * C + k] > 0.0 && sum > 0.0) ? (TP)(exp(logd(k) - top) / sum) : TP(0);
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_priors_workspace_bytes(int C, size_t* bytes) {
  RW_CHECK(bytes != nullptr && C >= 1 && C <= 255, RW_EINVAL, "bad sizes");
  *bytes = (size_t)3 * C * sizeof(double) + 256;
  return RW_OK;
}

int rw_priors_from_seeds(rw_graph h, const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C,
                         void* prior, int prior_dtype, void* work, size_t work_bytes, int32_t* status,
                         hipStream_t stream) {
  RW_CHECK(h != nullptr && seed_node != nullptr && seed_label != nullptr && prior != nullptr && work != nullptr &&
               status != nullptr,
           RW_EINVAL, "null argument");
  RW_CHECK(S >= 1 && C >= 1 && C <= 255, RW_EINVAL, "bad sizes (S = %lld, C = %d)", (long long)S, C);
  RW_CHECK(prior_dtype == RW_F64 || prior_dtype == RW_F32, RW_EINVAL, "priors are F64 or F32");
  size_t need = 0;
  RW_TRY(rw_priors_workspace_bytes(C, &need));
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "priors workspace too small: %zu < %zu", work_bytes, need);
  const Graph* g = &h->g;
  double* fit = static_cast<double*>(work);
  k_prior_fit<<<1, kFitThreads, 0, stream>>>(g->J, g->N, seed_node, seed_label, S, C, fit, status);
  RW_LAUNCH_CHECK();
  if (prior_dtype == RW_F64)
    k_prior_gauss<double><<<nblocks(g->N, 256), 256, 0, stream>>>(g->J, g->N, C, fit, static_cast<double*>(prior));
  else
    k_prior_gauss<float><<<nblocks(g->N, 256), 256, 0, stream>>>(g->J, g->N, C, fit, static_cast<float*>(prior));
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // extern "C"
