// Exact ("basic") random walker by Jacobi-preconditioned conjugate gradients in FP64 (Sec. II-A
// eq. (5) with gamma = 0): for every label k, L_n u_n^k = -B^T u_s^k.  All labels iterate together
// as a C x N block; scalars (alpha, beta) stay on the device, and the host reads the residual norms
// only every few iterations to test convergence.
#include <cmath>
#include <vector>

#include "rw_internal.h"

namespace rw {

constexpr int kCgBlocks = 512;     // partial-reduction blocks per label
constexpr int kCgCheckEvery = 8;   // iterations between host convergence checks

struct CgWork {
  uint8_t* map;
  uint8_t* anc;
  int64_t* seeds;
  int32_t* labels;
  double *r, *z, *p, *q;
  double* partial;   // kCgBlocks x C x 2
  double* sc;        // per label: [rz, pq, alpha, beta, rr, bb, rz_new, done]
};

static size_t cg_layout(const Graph* g, int C, int64_t S, void* base, CgWork* w) {
  Carver c(base);
  CgWork t;
  t.map = c.take<uint8_t>(g->N);
  t.anc = c.take<uint8_t>(g->N);
  t.seeds = c.take<int64_t>(std::max<int64_t>(S, 1));
  t.labels = c.take<int32_t>(std::max<int64_t>(S, 1));
  t.r = c.take<double>((size_t)C * g->N);
  t.z = c.take<double>((size_t)C * g->N);
  t.p = c.take<double>((size_t)C * g->N);
  t.q = c.take<double>((size_t)C * g->N);
  t.partial = c.take<double>((size_t)kCgBlocks * C * 2);
  t.sc = c.take<double>((size_t)C * 8);
  if (w) *w = t;
  return c.used;
}

__global__ void k_cg_clear_map(uint8_t* map, int64_t N) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) map[i] = 0;
}
__global__ void k_cg_set_map(uint8_t* map, const int64_t* seeds, const int32_t* labels, int64_t S) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < S) map[seeds[k]] = (uint8_t)(labels[k] + 1);
}

// sum of w_ij * v_j over neighbours j of i, with v given per node by a functor
template <typename F>
__device__ __forceinline__ double nbr_sum(const GridDev& G, const double* wgt, int64_t i, F v) {
  const int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / (G.nx * G.ny);
  double acc = 0.0;
  for (int d = 0; d < G.ndir; ++d) {
    if (head_in(G, x, y, z, d)) acc += wgt[d * G.N + i] * v(i + G.off[d]);
    if (tail_in(G, x, y, z, d)) acc += wgt[d * G.N + i - G.off[d]] * v(i - G.off[d]);
  }
  return acc;
}

// r = b - L_n x  (x zero on seeds); b_i = B(k, i) when an explicit right-hand side is given, else
// the seeded random walker's  b_i = sum over seed neighbours j with label k of w_ij  (= -B^T u_s)
__global__ void k_cg_init(GridDev G, const double* wgt, const double* deg, const uint8_t* map, int C, int x0_given,
                          const double* B, double* U, double* r) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (i >= G.N) return;
  double* x = U + (int64_t)k * G.N;
  if (map[i]) {
    r[(int64_t)k * G.N + i] = 0.0;
    return;
  }
  if (!x0_given) x[i] = 0.0;
  double b = B ? B[(int64_t)k * G.N + i] : nbr_sum(G, wgt, i, [&](int64_t j) { return map[j] == k + 1 ? 1.0 : 0.0; });
  double Ax = 0.0;
  if (x0_given) {
    Ax = deg[i] * x[i] - nbr_sum(G, wgt, i, [&](int64_t j) { return map[j] ? 0.0 : x[j]; });
  }
  r[(int64_t)k * G.N + i] = b - Ax;
}

// block partial sums of two products per label: s0 = a.b, s1 = c.d (fixed order)
__device__ __forceinline__ void block_reduce2(double v0, double v1, double* out0, double* out1) {
  __shared__ double s0[256], s1[256];
  s0[threadIdx.x] = v0;
  s1[threadIdx.x] = v1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out0 = s0[0];
    *out1 = s1[0];
  }
}

// z = r / d (non-seeds), partials of r.z and r.r
__global__ void k_cg_precond(int64_t N, const double* deg, const uint8_t* map, const double* r, double* z,
                             double* partial, int C) {
  int k = blockIdx.y;
  double rz = 0.0, rr = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = (int64_t)k * N + i;
    double ri = r[t];
    double zi = (map[i] || deg[i] <= 0.0) ? 0.0 : ri / deg[i];
    z[t] = zi;
    rz += ri * zi;
    rr += ri * ri;
  }
  block_reduce2(rz, rr, &partial[((int64_t)k * gridDim.x + blockIdx.x) * 2], &partial[((int64_t)k * gridDim.x + blockIdx.x) * 2 + 1]);
}

// scalars after the preconditioner: rz_new, rr; beta = rz_new / rz (0 on the first iteration)
__global__ void k_cg_scalars_rz(const double* partial, int nb, int C, double* sc, int first) {
  int k = threadIdx.x;
  if (k >= C) return;
  double rz = 0.0, rr = 0.0;
  for (int b = 0; b < nb; ++b) {
    rz += partial[((int64_t)k * nb + b) * 2];
    rr += partial[((int64_t)k * nb + b) * 2 + 1];
  }
  double* s = sc + 8 * k;
  if (first) s[5] = rr;                      // ||b||^2 (x0 = 0) or ||r0||^2
  s[3] = (first || s[0] == 0.0) ? 0.0 : rz / s[0];
  s[0] = rz;
  s[4] = rr;
}

// p = z + beta p
__global__ void k_cg_update_p(int64_t N, int C, const double* z, double* p, const double* sc) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (i >= N) return;
  int64_t t = (int64_t)k * N + i;
  p[t] = z[t] + sc[8 * k + 3] * p[t];
}

// q = L_n p (p zero on seeds), partial p.q
__global__ void k_cg_apply(GridDev G, const double* wgt, const double* deg, const uint8_t* map, const double* p,
                           double* q, double* partial) {
  int k = blockIdx.y;
  const double* pk = p + (int64_t)k * G.N;
  double pq = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G.N; i += (int64_t)gridDim.x * blockDim.x) {
    double qi = 0.0;
    if (!map[i]) {
      qi = deg[i] * pk[i] - nbr_sum(G, wgt, i, [&](int64_t j) { return map[j] ? 0.0 : pk[j]; });
      pq += pk[i] * qi;
    }
    q[(int64_t)k * G.N + i] = qi;
  }
  block_reduce2(pq, 0.0, &partial[((int64_t)k * gridDim.x + blockIdx.x) * 2], &partial[((int64_t)k * gridDim.x + blockIdx.x) * 2 + 1]);
}

__global__ void k_cg_scalars_pq(const double* partial, int nb, int C, double* sc) {
  int k = threadIdx.x;
  if (k >= C) return;
  double pq = 0.0;
  for (int b = 0; b < nb; ++b) pq += partial[((int64_t)k * nb + b) * 2];
  double* s = sc + 8 * k;
  s[1] = pq;
  s[2] = (pq != 0.0 && s[0] != 0.0) ? s[0] / pq : 0.0;
}

// x += alpha p, r -= alpha q
__global__ void k_cg_axpy(int64_t N, double* U, double* r, const double* p, const double* q, const double* sc) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (i >= N) return;
  int64_t t = (int64_t)k * N + i;
  double a = sc[8 * k + 2];
  U[t] += a * p[t];
  r[t] -= a * q[t];
}

// seed rows: one-hot (random walker) or zero (explicit right-hand side: the adjoint vanishes there)
__global__ void k_cg_finish(int64_t N, const uint8_t* map, int onehot, double* U) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (i >= N) return;
  if (map[i]) U[(int64_t)k * N + i] = (onehot && map[i] - 1 == k) ? 1.0 : 0.0;
}

static int cg_core(rw_graph h, const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C,
                   const double* B, double tol, int max_iter, int x0_given, double* U, void* work, size_t work_bytes,
                   hipStream_t stream, rw_cg_info* info) {
  RW_CHECK(h != nullptr && U != nullptr && work != nullptr, RW_EINVAL, "null argument");
  const Graph* g = &h->g;
  RW_CHECK(g->dtype == RW_F64, RW_EINVAL, "the CG solver needs an FP64 graph");
  RW_CHECK(C >= 1 && C <= 255, RW_EINVAL, "C must be in [1, 255]");
  RW_CHECK(S >= 1 && seed_node != nullptr && seed_label != nullptr, RW_EINVAL, "at least one seed is required");
  RW_CHECK(tol > 0.0 && max_iter >= 1, RW_EINVAL, "tol > 0 and max_iter >= 1 required");
  // sort / validate seeds on the host
  std::vector<std::pair<int64_t, int32_t>> v((size_t)S);
  for (int64_t k = 0; k < S; ++k) {
    RW_CHECK(seed_node[k] >= 0 && seed_node[k] < g->N, RW_EINVAL, "seed node out of range");
    RW_CHECK(seed_label[k] >= 0 && seed_label[k] < C, RW_EINVAL, "seed label out of range");
    v[k] = {seed_node[k], seed_label[k]};
  }
  std::sort(v.begin(), v.end());
  std::vector<int64_t> nodes;
  std::vector<int32_t> labels;
  for (size_t k = 0; k < v.size(); ++k) {
    if (k && v[k].first == v[k - 1].first) {
      RW_CHECK(v[k].second == v[k - 1].second, RW_EINVAL, "conflicting labels on node %lld", (long long)v[k].first);
      continue;
    }
    nodes.push_back(v[k].first);
    labels.push_back(v[k].second);
  }
  const int64_t Sd = (int64_t)nodes.size();
  CgWork w;
  size_t need = cg_layout(g, C, g->N, work, &w);
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "cg workspace too small: %zu < %zu", work_bytes, need);
  RW_HIP(hipMemcpyAsync(w.seeds, nodes.data(), Sd * sizeof(int64_t), hipMemcpyHostToDevice, stream));
  RW_HIP(hipMemcpyAsync(w.labels, labels.data(), Sd * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  RW_TRY(check_anchored(&h->g, w.seeds, Sd, w.anc, stream));
  const int64_t N = g->N;
  const GridDev G = grid_of(g);
  const double* wgt = static_cast<const double*>(g->weight);
  k_cg_clear_map<<<nblocks(N, 256), 256, 0, stream>>>(w.map, N);
  k_cg_set_map<<<nblocks(Sd, 256), 256, 0, stream>>>(w.map, w.seeds, w.labels, Sd);
  RW_LAUNCH_CHECK();
  dim3 gridN(nblocks(N, 256), C);
  const int nbk = (int)std::min<int64_t>(kCgBlocks, nblocks(N, 256));
  dim3 gridR(nbk, C);
  k_cg_init<<<gridN, 256, 0, stream>>>(G, wgt, g->degree, w.map, C, x0_given, B, U, w.r);
  RW_LAUNCH_CHECK();
  k_cg_precond<<<gridR, 256, 0, stream>>>(N, g->degree, w.map, w.r, w.z, w.partial, C);
  k_cg_scalars_rz<<<1, 256, 0, stream>>>(w.partial, nbk, C, w.sc, 1);
  RW_HIP(hipMemsetAsync(w.p, 0, (size_t)C * N * sizeof(double), stream));
  k_cg_update_p<<<gridN, 256, 0, stream>>>(N, C, w.z, w.p, w.sc);
  RW_LAUNCH_CHECK();
  std::vector<double> sc((size_t)8 * C);
  RW_HIP(hipMemcpyAsync(sc.data(), w.sc, sc.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
  RW_HIP(hipStreamSynchronize(stream));
  std::vector<double> bb(C);
  for (int k = 0; k < C; ++k) bb[k] = sc[8 * k + 5];
  auto converged = [&](double* worst) {
    bool all = true;
    *worst = 0.0;
    for (int k = 0; k < C; ++k) {
      double rel = bb[k] > 0.0 ? std::sqrt(sc[8 * k + 4] / bb[k]) : 0.0;
      *worst = std::max(*worst, rel);
      if (rel > tol) all = false;
    }
    return all;
  };
  double worst = 0.0;
  int it = 0;
  bool done = converged(&worst);
  while (!done && it < max_iter) {
    k_cg_apply<<<gridR, 256, 0, stream>>>(G, wgt, g->degree, w.map, w.p, w.q, w.partial);
    k_cg_scalars_pq<<<1, 256, 0, stream>>>(w.partial, nbk, C, w.sc);
    k_cg_axpy<<<gridN, 256, 0, stream>>>(N, U, w.r, w.p, w.q, w.sc);
    k_cg_precond<<<gridR, 256, 0, stream>>>(N, g->degree, w.map, w.r, w.z, w.partial, C);
    k_cg_scalars_rz<<<1, 256, 0, stream>>>(w.partial, nbk, C, w.sc, 0);
    k_cg_update_p<<<gridN, 256, 0, stream>>>(N, C, w.z, w.p, w.sc);
    RW_LAUNCH_CHECK();
    ++it;
    if (it % kCgCheckEvery == 0 || it == max_iter) {
      RW_HIP(hipMemcpyAsync(sc.data(), w.sc, sc.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
      RW_HIP(hipStreamSynchronize(stream));
      done = converged(&worst);
    }
  }
  k_cg_finish<<<gridN, 256, 0, stream>>>(N, w.map, B ? 0 : 1, U);
  RW_LAUNCH_CHECK();
  RW_HIP(hipStreamSynchronize(stream));
  if (info) {
    info->iters = it;
    info->rel_residual = worst;
  }
  if (!done) {
    set_error("CG: relative residual %.3g > %.3g after %d iterations", worst, tol, it);
    return RW_ENOCONV;
  }
  return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_cg_workspace_bytes(rw_graph h, int C, size_t* bytes) {
  RW_CHECK(h != nullptr && bytes != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(C >= 1 && C <= 255, RW_EINVAL, "C must be in [1, 255]");
  *bytes = cg_layout(&h->g, C, h->g.N, nullptr, nullptr);
  return RW_OK;
}

int rw_cg_solve(rw_graph h, const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C, double tol,
                int max_iter, int x0_given, double* U, void* work, size_t work_bytes, hipStream_t stream,
                rw_cg_info* info) {
  RW_NOT_CAPTURING(stream);
  return cg_core(h, seed_node, seed_label, S, C, nullptr, tol, max_iter, x0_given, U, work, work_bytes, stream, info);
}

int rw_cg_solve_rhs(rw_graph h, const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C, const double* B,
                    double tol, int max_iter, int x0_given, double* X, void* work, size_t work_bytes,
                    hipStream_t stream, rw_cg_info* info) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(B != nullptr, RW_EINVAL, "null right-hand side");
  return cg_core(h, seed_node, seed_label, S, C, B, tol, max_iter, x0_given, X, work, work_bytes, stream, info);
}

}  // extern "C"
