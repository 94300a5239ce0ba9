// Matrix-free stencil operator: Y = alpha * op(X) + beta * X + gamma * Z for a column-major N x b
// block, op = L_hat = I - D^{-1/2} W D^{-1/2} (zero rows where d = 0) or L = D - W (Sec. II-A, Sec. II-C).
//
// Per node the operator needs the diagonal and the coefficients of its 4/8/6 incident edges:
// forward edges are stored at the node, backward ones at the neighbour (the edge's tail).  One
// thread owns one node, loads its coefficients once and sweeps every column of the block, so the
// coefficient planes are read once per launch while X and Y stream through.
#include "rw_internal.h"

namespace rw {

template <typename T, int NDIR>
struct StencilArgs {
  GridDev G;
  const T* X;
  T* Y;
  const T* Z;
  const T* coef;
  const T* diag;
  int64_t b;
  typename Elem<T>::C alpha, beta, gamma;
};

template <typename T, int NDIR>
__global__ __launch_bounds__(256) void k_stencil(StencilArgs<T, NDIR> a) {
  using C = typename Elem<T>::C;
  const GridDev& G = a.G;
  const int64_t x = blockIdx.x * (int64_t)64 + threadIdx.x;
  const int64_t r = blockIdx.y * (int64_t)4 + threadIdx.y;  // row index y + ny*z
  if (x >= G.nx || r >= G.ny * G.nz) return;
  const int64_t y = r % G.ny, z = r / G.ny;
  const int64_t i = x + G.nx * r;
  C c[2 * NDIR];
  int64_t nb[2 * NDIR];
#pragma unroll
  for (int d = 0; d < NDIR; ++d) {
    bool f = head_in(G, x, y, z, d);
    c[d] = f ? (C)a.coef[d * G.N + i] : C(0);
    nb[d] = f ? i + G.off[d] : i;
    bool t = tail_in(G, x, y, z, d);
    c[NDIR + d] = t ? (C)a.coef[d * G.N + i - G.off[d]] : C(0);
    nb[NDIR + d] = t ? i - G.off[d] : i;
  }
  const C dg = (C)a.diag[i];
  const C al = a.alpha, be = a.beta, ga = a.gamma;
  for (int64_t col = 0; col < a.b; ++col) {
    const T* xc = a.X + col * G.N;
    C xi = (C)xc[i];
    C acc = dg * xi;
#pragma unroll
    for (int k = 0; k < 2 * NDIR; ++k) acc -= c[k] * (C)xc[nb[k]];
    C out = al * acc;
    if (be != C(0)) out += be * xi;
    if (a.Z != nullptr) out += ga * (C)a.Z[col * G.N + i];
    a.Y[col * G.N + i] = (T)out;
  }
}

template <typename T, int NDIR>
static int launch(const Graph* g, const void* X, void* Y, const void* Z, int64_t b, double alpha,
                  double beta, double gamma, hipStream_t s) {
  using C = typename Elem<T>::C;
  StencilArgs<T, NDIR> a;
  a.G = grid_of(g);
  a.X = static_cast<const T*>(X);
  a.Y = static_cast<T*>(Y);
  a.Z = gamma != 0.0 ? static_cast<const T*>(Z) : nullptr;
  a.coef = static_cast<const T*>(g->coef);
  a.diag = static_cast<const T*>(g->diag);
  a.b = b;
  a.alpha = (C)alpha;
  a.beta = (C)beta;
  a.gamma = (C)gamma;
  dim3 block(64, 4);
  dim3 grid(nblocks(g->nx, 64), nblocks(g->ny * g->nz, 4));
  k_stencil<T, NDIR><<<grid, block, 0, s>>>(a);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

int stencil_apply(const Graph* g, const void* X, void* Y, const void* Z, int64_t b, double alpha,
                  double beta, double gamma, hipStream_t s) {
  if (b <= 0) return RW_OK;
  RW_CHECK(g->ny * g->nz < (int64_t)4 * 65535, RW_EINVAL, "grid too tall for the stencil launch");
  if (g->dtype == RW_F64) {
    switch (g->ndir) {
      case 2: return launch<double, 2>(g, X, Y, Z, b, alpha, beta, gamma, s);
      case 3: return launch<double, 3>(g, X, Y, Z, b, alpha, beta, gamma, s);
      default: return launch<double, 4>(g, X, Y, Z, b, alpha, beta, gamma, s);
    }
  }
  switch (g->ndir) {
    case 2: return launch<float, 2>(g, X, Y, Z, b, alpha, beta, gamma, s);
    case 3: return launch<float, 3>(g, X, Y, Z, b, alpha, beta, gamma, s);
    default: return launch<float, 4>(g, X, Y, Z, b, alpha, beta, gamma, s);
  }
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_apply_laplacian(rw_graph h, const void* X, void* Y, int64_t b, hipStream_t stream) {
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  RW_CHECK(b >= 0, RW_EINVAL, "b must be >= 0");
  RW_CHECK(b == 0 || (X != nullptr && Y != nullptr), RW_EINVAL, "null X or Y");
  RW_CHECK(X != Y || b == 0, RW_EINVAL, "X and Y must be distinct");
  return stencil_apply(&h->g, X, Y, nullptr, b, 1.0, 0.0, 0.0, stream);
}

int rw_apply_laplacian_axpby(rw_graph h, const void* X, void* Y, const void* Z, int64_t b, double alpha,
                             double beta, double gamma, hipStream_t stream) {
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  RW_CHECK(b >= 0, RW_EINVAL, "b must be >= 0");
  RW_CHECK(b == 0 || (X != nullptr && Y != nullptr), RW_EINVAL, "null X or Y");
  RW_CHECK(X != Y || b == 0, RW_EINVAL, "X and Y must be distinct");
  RW_CHECK(gamma == 0.0 || Z != nullptr, RW_EINVAL, "Z required when gamma != 0");
  return stencil_apply(&h->g, X, Y, Z, b, alpha, beta, gamma, stream);
}

}  // extern "C"
