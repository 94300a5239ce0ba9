// Offline eigenpairs of the graph operator (Sec. II-B eq. (6): the m smallest, null pair included)
// and their online update after graph edits (Sec. III-B eqs. (26)-(28), plus Rayleigh-Ritz).
//
// Eigensolver: block Chebyshev-filtered subspace iteration with Rayleigh-Ritz.  The known null
// vector (eigenvalue 0) is deflated analytically: the block lives in its orthogonal complement and
// the null vector is written as column 0 of Q.  Each outer iteration applies a degree-d Chebyshev
// polynomial of the operator that damps [a, b] (b = 2 for L_hat, the Gershgorin bound 2 max d for L),
// i.e. d fused stencil passes over the block, then one Rayleigh-Ritz step: G = F^T F and H = F^T op F
// in FP64, W with F W orthonormal, eig(W^T H W) = Z Theta Z^T, X = F W Z.  All dense work is FP64; the
// block itself is in the graph's type.  On MI355X the cost is dominated by the HBM-bound stencil
// passes, which the polynomial filter amortizes over one FP64 Gram / eigendecomposition per outer
// iteration.
//   * a: the block's largest Ritz value.  Next to a warm block (an update) the random guard columns hold
//     it near 1 at first, and the low-degree filter on [a, b] turns them into the low-frequency directions
//     the warm columns need; a tighter estimate of the top of the guard band leaves the guards random and
//     gains only about 3x per 64 passes for the top wanted columns of the 512 x 512 workload (their gap to
//     the band is 4e-4 of a spectrum of width 2), measured slower for every update.
//   * soft locking: the leading wanted columns whose residuals are below tol / 4 are not filtered (they
//     stay in the Rayleigh-Ritz step), so the filter's cost follows the unconverged columns.
//   * degree: enough for the largest residual among the filtered wanted columns to fall to tol / 8 at
//     the gain of the lowest filtered Ritz value, between 4 and 64 (at most the amplification of a cold
//     start, 1e4 in FP32 and 1e8 in FP64).
#include <chrono>
#include <cmath>
#include <vector>

#include "rw_internal.h"

namespace rw {

struct EigWork {
  char* B[4];
  double *G, *G2, *V, *s, *W, *H, *T, *Hp, *Z, *WZ, *theta, *res, *cq, *syw, *tmp, *partial;
  int* info;
};

static int guard_of(int m, const rw_eig_opts* o) {
  if (o && o->guard > 0) return o->guard;
  return std::max(8, (m + 9) / 10);
}

static size_t eig_layout(const Graph* g, int nb, void* base, EigWork* w) {
  Carver c(base);
  size_t es = dtype_size(g->dtype);
  EigWork t;
  for (int k = 0; k < 4; ++k) t.B[k] = c.take<char>((size_t)g->N * nb * es);
  size_t n2 = (size_t)nb * nb;
  t.G = c.take<double>(n2); t.V = c.take<double>(n2); t.W = c.take<double>(n2); t.H = c.take<double>(n2);
  t.T = c.take<double>(n2); t.Hp = c.take<double>(n2); t.Z = c.take<double>(n2); t.WZ = c.take<double>(n2);
  t.G2 = c.take<double>(n2);
  t.syw = c.take<double>(std::max(syev_work_count(nb, 1, true, 0), tridiag_fits(nb) ? tridiag_work_count(nb) : 0));
  t.s = c.take<double>(nb); t.theta = c.take<double>(nb); t.res = c.take<double>(nb); t.cq = c.take<double>(nb);
  t.tmp = c.take<double>(std::max(nb, 16));
  size_t pc = std::max({gram_partial_count(g->N, nb, nb), norm_partial_count(nb), gram_partial_count(g->N, 1, nb),
                       rotate_pair_partial_count(nb)});
  t.partial = c.take<double>(pc);
  t.info = c.take<int>(16);
  if (w) *w = t;
  return c.used;
}

// W(:, j) = V(:, j) / sqrt(max(s_j, floor_rel * s_max)),  s ascending (s_max = s[n-1])
__global__ void k_scale_cols(const double* V, const double* s, double* W, int n, double floor_rel) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  int j = (int)(t / n);
  double smax = fmax(s[n - 1], 1e-300);
  double sj = fmax(s[j], floor_rel * smax);
  W[t] = V[t] / sqrt(sj);
}

// E = G - I and max |E_ij| (out[0] zeroed beforehand; blocks combine their maxima with an integer max on
// the bit patterns, which orders non-negative doubles like their values, so the result does not depend on
// the order).  With PROJ, G is first formed as the projected Gram from Gq (as k_gram_project does, also
// writing G and c).
template <bool PROJ>
__global__ __launch_bounds__(256) void k_offI_absmax(const double* Gin, int n, double* E, double* out,
                                                     double* Gout = nullptr, double* cvec = nullptr) {
  __shared__ double red[4];
  double m = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)n * n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % n), j = (int)(t / n);
    double gv;
    if (PROJ) {
      const double ci = Gin[i + 1], cj = Gin[j + 1];
      gv = Gin[(int64_t)(j + 1) * (n + 1) + i + 1] - (2.0 - Gin[0]) * ci * cj;
      Gout[t] = gv;
      if (j == 0) cvec[i] = ci;
    } else {
      gv = Gin[t];
    }
    const double e = gv - (i == j ? 1.0 : 0.0);
    E[t] = e;
    m = fmax(m, fabs(e));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    atomicMax(reinterpret_cast<unsigned long long*>(out), (unsigned long long)__double_as_longlong(r));
  }
}

// W = G^{-1/2} = I - E/2 + (3/8) E^2 + O(|E|^3) for G = I + E (E2 = E E)
__global__ void k_series_w(const double* E, const double* E2, double* W, int n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t % n), j = (int)(t / n);
  W[t] = (i == j ? 1.0 : 0.0) - 0.5 * E[t] + 0.375 * E2[t];
}

// Gram of the projected block F = Qv - g c^T (c = Qv^T g, g of unit norm) from Gq = Q^T Q of Q = [g, Qv]
// ((nb + 1)^2): F^T F = Qv^T Qv - (2 - g^T g) c c^T; also returns c
__global__ void k_gram_project(const double* Gq, int nb, double* G, double* cvec) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nb * nb) return;
  const int i = (int)(t % nb), j = (int)(t / nb), n1 = nb + 1;
  const double ci = Gq[i + 1], cj = Gq[j + 1];
  G[t] = Gq[(int64_t)(j + 1) * n1 + i + 1] - (2.0 - Gq[0]) * ci * cj;
  if (j == 0) cvec[i] = ci;
}

// rotation of the projected block through Q = [g, Qv]: F V = Q V' with V' ((nb + 1) x nb, ld nb + 1)
// holding -(c^T V) in row 0 and V below; one wave per column
__global__ __launch_bounds__(64) void k_fold_rows(const double* V, const double* cvec, int nb, double* Vp) {
  const int j = blockIdx.x, lane = threadIdx.x;
  const double* vj = V + (int64_t)j * nb;
  double* out = Vp + (int64_t)j * (nb + 1);
  double acc = 0.0;
  for (int i = lane; i < nb; i += 64) {
    const double x = vj[i];
    acc += cvec[i] * x;
    out[i + 1] = x;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) out[0] = -acc;
}

__global__ void k_symmetrize(double* A, int n) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  int i = (int)(t % n), j = (int)(t / n);
  if (i < j) {
    double v = 0.5 * (A[t] + A[j + (int64_t)i * n]);
    A[t] = v;
    A[j + (int64_t)i * n] = v;
  }
}

// copy column block src (rows x cols, ld_s) into dst (ld_d), with type conversion
static int copy_cols(int dts, const void* src, int64_t lds, int dtd, void* dst, int64_t ldd, int64_t rows, int cols,
                     hipStream_t s) {
  return convert_block(dts, src, lds, dtd, dst, ldd, rows, cols, s);
}

struct Ctx {
  const Graph* g;
  int dt;
  int64_t N;
  EigWork w;
  hipStream_t s;
  int64_t spmm_cols = 0;
  double floor_rel;
};

__global__ void k_copy_d(const double* a, double* b, int64_t n) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t];
}

// One Rayleigh-Ritz step on the block F (nb columns).  Outputs X = F W Z, theta and res (the residual
// norms of X's columns); LX is scratch for op X, which no caller reads afterwards.
// W makes F W orthonormal: W = R^{-1} from the Cholesky factor of G = F^T F (Cholesky QR), or, if
// G is numerically singular, W = V s^{-1/2} from its eigendecomposition with small s floored.  With
// `near_orth` (F already orthonormal up to storage rounding, as a stored eigenbasis is) and
// max |G - I| < 1e-4, W = G^{-1/2} from its series I - E/2 + 3/8 E^2 (truncation below 1e-12).
static int rr_step(Ctx& c, int nb, char* F, char* LF, char* X, char* LX, bool near_orth = false,
                   bool fold = false) {
  const Graph* g = c.g;
  EigWork& w = c.w;
  const int64_t n2 = (int64_t)nb * nb;
  // with `fold`, the column before F holds the null vector g and the block is the projection F - g (g^T F):
  // the projection enters through the Gram of [g, F] and the rotation's extra row, and op F serves for
  // op of the projected block (op g = 0).  X may then be F itself (in-place rotation).
  char* Q0 = F - dtype_size(c.dt) * c.N;
  // a nearly orthonormal block (the update path) allows FP32 accumulation over row chunks
  if (fold) {
    RW_TRY(gram(c.dt, Q0, c.N, Q0, c.N, c.N, nb + 1, nb + 1, w.Hp, w.partial, c.s, true, near_orth));
    if (!near_orth) {
      k_gram_project<<<nblocks(n2, 256), 256, 0, c.s>>>(w.Hp, nb, w.G, w.cq);
      RW_LAUNCH_CHECK();
    }
  } else {
    RW_TRY(gram(c.dt, F, c.N, F, c.N, c.N, nb, nb, w.G, w.partial, c.s, true, near_orth));
  }
  // W from the series is formed without waiting for max |G - I|: that value is read with the eigensolver's
  // flag, and when it is too large for the series the projected matrix is formed again with Cholesky QR
  const double* offI = nullptr;
  bool have_w = false;
  if (near_orth) {
    RW_HIP(hipMemsetAsync(w.tmp, 0, sizeof(double), c.s));
    const unsigned nbk = (unsigned)std::min<int64_t>(nblocks(n2, 256), 160);
    if (fold) k_offI_absmax<true><<<nbk, 256, 0, c.s>>>(w.Hp, nb, w.G2, w.tmp, w.G, w.cq);
    else k_offI_absmax<false><<<nbk, 256, 0, c.s>>>(w.G, nb, w.G2, w.tmp);
    RW_LAUNCH_CHECK();
    RW_TRY(gram(RW_F64, w.G2, nb, w.G2, nb, nb, nb, nb, w.V, w.partial, c.s, true));   // E^2 = E^T E (E symmetric)
    k_series_w<<<nblocks(n2, 256), 256, 0, c.s>>>(w.G2, w.V, w.W, nb);
    RW_LAUNCH_CHECK();
    offI = w.tmp;
    have_w = true;
  }
  // W = R^{-1} of Cholesky QR, or from the eigendecomposition of G when that fails
  auto cholesky_w = [&]() -> int {
    k_copy_d<<<nblocks(n2, 256), 256, 0, c.s>>>(w.G, w.G2, n2);
    RW_LAUNCH_CHECK();
    RW_TRY(chol_inverse(w.G2, w.W, nb, w.info, c.s));
    int bad = 0;
    RW_HIP(hipMemcpyAsync(&bad, w.info, sizeof(int), hipMemcpyDeviceToHost, c.s));
    RW_HIP(hipStreamSynchronize(c.s));
    if (bad != 0) {
      RW_TRY(syev_batched(w.G, w.s, w.V, nullptr, 0, nb, 1, w.syw, c.s));
      k_scale_cols<<<nblocks(n2, 256), 256, 0, c.s>>>(w.V, w.s, w.W, nb, c.floor_rel);
      RW_LAUNCH_CHECK();
    }
    return RW_OK;
  };
  if (!have_w) RW_TRY(cholesky_w());
  RW_TRY(stencil_apply(g, F, LF, nullptr, nb, 1.0, 0.0, 0.0, c.s));
  c.spmm_cols += nb;
  RW_TRY(gram(c.dt, F, c.N, LF, c.N, c.N, nb, nb, w.H, w.partial, c.s, true, near_orth));
  // with an FP32 or BF16 basis the projected matrix carries errors near 1e-7 relative: the tridiagonal
  // solver (Householder, bisection, inverse iteration) serves when its eigenvalues are separated, else
  // Jacobi, whose rotations below 1e-10 relative change nothing the rotated basis can represent
  int est = RW_ENOCONV;
  for (;;) {
    RW_TRY(gram(RW_F64, w.H, nb, w.W, nb, nb, nb, nb, w.T, w.partial, c.s));         // T = H^T W = H W
    RW_TRY(gram(RW_F64, w.W, nb, w.T, nb, nb, nb, nb, w.Hp, w.partial, c.s));        // Hp = W^T H W
    k_symmetrize<<<nblocks((int64_t)nb * nb, 256), 256, 0, c.s>>>(w.Hp, nb);
    RW_LAUNCH_CHECK();
    est = RW_ENOCONV;
    const double* tri_flag = nullptr;
    if (c.dt != RW_F64 && tridiag_fits(nb)) {
      est = syev_tridiag(w.Hp, w.theta, w.Z, nb, w.syw, c.s, offI != nullptr ? &tri_flag : nullptr);
      if (est != RW_OK && est != RW_ENOCONV) return est;
    }
    if (offI == nullptr) break;
    void* stage = nullptr;
    RW_TRY(host_stage(2 * sizeof(double), &stage));
    double* hs = static_cast<double*>(stage);
    hs[1] = 0.0;
    RW_HIP(hipMemcpyAsync(hs, offI, sizeof(double), hipMemcpyDeviceToHost, c.s));
    if (tri_flag != nullptr) RW_HIP(hipMemcpyAsync(hs + 1, tri_flag, sizeof(double), hipMemcpyDeviceToHost, c.s));
    RW_HIP(hipStreamSynchronize(c.s));
    const double e = hs[0], fl = hs[1];
    if (tri_flag != nullptr && fl != 0.0) est = RW_ENOCONV;
    offI = nullptr;
    if (e < 1e-4) break;
    have_w = false;   // the series does not apply: Cholesky QR, then the projected matrix again
    RW_TRY(cholesky_w());
  }
  if (est == RW_ENOCONV)
    RW_TRY(syev_batched(w.Hp, w.theta, w.Z, nullptr, 0, nb, 1, w.syw, c.s, c.dt == RW_F64 ? 0.0 : 1e-10));
  if (have_w)   // the series W is symmetric: W Z = W^T Z on the matrix cores
    RW_TRY(gram(RW_F64, w.W, nb, w.Z, nb, nb, nb, nb, w.WZ, w.partial, c.s));
  else
    RW_TRY(gemm_tn(RW_F64, w.W, nb, w.Z, nb, w.WZ, nb, nb, nb, nb, 0.0, c.s));    // WZ = W Z
  if (fold) {
    k_fold_rows<<<nb, 64, 0, c.s>>>(w.WZ, w.cq, nb, w.T);
    RW_LAUNCH_CHECK();
  }
  const double* Vr = fold ? w.T : w.WZ;   // the rotation, acting on [g, F] when folded
  const int kr = fold ? nb + 1 : nb;
  if (rotate_pair_fits(c.dt, c.N, kr, nb)) {   // X and the residual norms in one pass (op X not stored)
    RW_TRY(rotate_pair((const float*)(fold ? Q0 : F), (const float*)LF, fold ? 1 : 0, c.N, Vr, kr, w.theta,
                       (float*)X, nullptr, c.N, kr, nb, w.res, w.partial, c.s));
    return RW_OK;
  }
  RW_TRY(gemm_tn(c.dt, fold ? Q0 : F, c.N, Vr, kr, X, c.N, c.N, kr, nb, 0.0, c.s));   // X = (F - g c^T) W Z
  RW_TRY(gemm_tn(c.dt, LF, c.N, w.WZ, nb, LX, c.N, c.N, nb, nb, 0.0, c.s));      // op X
  RW_TRY(residual_norms(c.dt, LX, X, w.theta, c.N, nb, c.N, w.res, w.partial, c.s));
  return RW_OK;
}

static double upper_bound(const Graph* g, EigWork& w, hipStream_t s, int* st) {
  *st = RW_OK;
  if (g->normalized) return 2.0;
  if ((*st = absmax(g->degree, g->N, w.tmp, s)) != RW_OK) return 0.0;
  double dmax = 0.0;
  if (hipMemcpyAsync(&dmax, w.tmp, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("reading the degree bound failed");
    *st = RW_EHIP;
  }
  return 2.0 * dmax * 1.0000001 + 1e-300;
}

// Chebyshev-filtered subspace iteration.  On entry block B[0] holds the start vectors (nb columns).
static int chfsi(Ctx& c, int m, int nb, const rw_eig_opts* o, void* Q, double* lambda, rw_eig_info* info) {
  const Graph* g = c.g;
  EigWork& w = c.w;
  const int k = m - 1;
  int st = RW_OK;
  const double bup = upper_bound(g, w, c.s, &st);
  RW_TRY(st);
  RW_TRY(project_out(c.dt, w.B[0], c.N, g->ghat, c.N, nb, w.tmp, w.partial, c.s));
  int ix = 2, ilx = 3;
  RW_TRY(rr_step(c, nb, w.B[0], w.B[1], w.B[ix], w.B[ilx]));
  std::vector<double> th(nb), rs(nb);
  const double amp_target = c.dt == RW_F64 ? 1e8 : 1e4;
  int it = 0;
  int nconv = 0;
  double maxres = INFINITY;
  const int max_iter = o->max_iter > 0 ? o->max_iter : 200;
  for (;;) {
    RW_HIP(hipMemcpyAsync(th.data(), w.theta, nb * sizeof(double), hipMemcpyDeviceToHost, c.s));
    RW_HIP(hipMemcpyAsync(rs.data(), w.res, nb * sizeof(double), hipMemcpyDeviceToHost, c.s));
    RW_HIP(hipStreamSynchronize(c.s));
    nconv = 0;
    maxres = 0.0;
    for (int j = 0; j < k; ++j) {
      maxres = std::max(maxres, rs[j]);
      if (rs[j] <= o->tol) ++nconv;
    }
    if (nconv == k || it >= max_iter) break;
    ++it;
    // soft locking: the leading wanted columns well below tol are left out of the filter
    int nlock = 0;
    while (nlock < k && rs[nlock] <= 0.25 * o->tol) ++nlock;
    double res_act = 0.0;
    for (int j = nlock; j < k; ++j) res_act = std::max(res_act, rs[j]);
    // filter bounds
    double a = th[nb - 1], a0 = std::max(th[nlock], 0.0);
    if (!(a < bup)) a = 0.5 * bup;
    if (!(a0 < a)) a0 = 0.0;
    const double e = 0.5 * (bup - a), cc = 0.5 * (bup + a);
    int deg = o->degree;
    if (deg <= 0) {
      double t0 = (cc - a0) / e;
      double ac = t0 > 1.0 ? std::acosh(t0) : 1e-3;
      const double amp = std::min(amp_target, std::max(16.0, 8.0 * res_act / o->tol));
      deg = (int)std::ceil(std::acosh(amp) / ac);
      deg = std::min(64, std::max(4, deg));
    }
    const int nfl = nb - nlock;                // filtered columns nlock .. nb-1
    const size_t off = dtype_size(c.dt) * (size_t)c.N * nlock;
    // buffers: Y0 = X, Y1, Y2 free
    int b0 = ix, b1 = -1, b2 = -1;
    {
      int fr[3], nf = 0;
      for (int q = 0; q < 4; ++q)
        if (q != ix) fr[nf++] = q;
      b1 = fr[0];
      b2 = fr[1];
    }
    double sigma = e / (a0 - cc);
    const double tau = 2.0 / sigma;
    const int bx = ix;   // the Ritz block X (the locked columns are taken from it)
    // Y1 = (op X - c X) sigma / e
    RW_TRY(stencil_apply(g, w.B[b0] + off, w.B[b1] + off, nullptr, nfl, sigma / e, -cc * sigma / e, 0.0, c.s));
    c.spmm_cols += nfl;
    for (int i = 2; i <= deg; ++i) {
      double sn = 1.0 / (tau - sigma);
      // Y2 = (op Y1 - c Y1) 2 sn / e - sigma sn Y0
      RW_TRY(stencil_apply(g, w.B[b1] + off, w.B[b2] + off, w.B[b0] + off, nfl, 2.0 * sn / e, -2.0 * cc * sn / e,
                           -sigma * sn, c.s));
      c.spmm_cols += nfl;
      int t = b0;
      b0 = b1;
      b1 = b2;
      b2 = t;
      sigma = sn;
    }
    // filtered columns in b1; the locked ones join them unfiltered; the other three buffers are free
    if (nlock > 0 && b1 != bx) RW_TRY(copy_cols(c.dt, w.B[bx], c.N, c.dt, w.B[b1], c.N, c.N, nlock, c.s));
    RW_TRY(project_out(c.dt, w.B[b1] + off, c.N, g->ghat, c.N, nfl, w.tmp, w.partial, c.s));
    int fr[3], nf = 0;
    for (int q = 0; q < 4; ++q)
      if (q != b1) fr[nf++] = q;
    RW_TRY(rr_step(c, nb, w.B[b1], w.B[fr[0]], w.B[fr[1]], w.B[fr[2]]));
    ix = fr[1];
    ilx = fr[2];
  }
  // final clean-up Rayleigh-Ritz on the converged block (restores orthonormality to working precision)
  {
    int fr[3], nf = 0;
    for (int q = 0; q < 4; ++q)
      if (q != ix) fr[nf++] = q;
    RW_TRY(rr_step(c, nb, w.B[ix], w.B[fr[0]], w.B[fr[1]], w.B[fr[2]]));
    ix = fr[1];
    RW_HIP(hipMemcpyAsync(rs.data(), w.res, nb * sizeof(double), hipMemcpyDeviceToHost, c.s));
    RW_HIP(hipStreamSynchronize(c.s));
    nconv = 0;
    maxres = 0.0;
    for (int j = 0; j < k; ++j) {
      maxres = std::max(maxres, rs[j]);
      if (rs[j] <= o->tol) ++nconv;
    }
  }
  // outputs: Q = [ghat, X(:, 0:k)], lambda = [0, theta(0:k)]
  const int qdt = o->q_dtype;
  RW_TRY(copy_cols(c.dt, g->ghat, c.N, qdt, Q, c.N, c.N, 1, c.s));
  RW_TRY(copy_cols(c.dt, w.B[ix], c.N, qdt, (char*)Q + dtype_size(qdt) * c.N, c.N, c.N, k, c.s));
  const double zero = 0.0;
  RW_HIP(hipMemcpyAsync(lambda, &zero, sizeof(double), hipMemcpyHostToDevice, c.s));
  RW_HIP(hipMemcpyAsync(lambda + 1, w.theta, k * sizeof(double), hipMemcpyDeviceToDevice, c.s));
  RW_HIP(hipStreamSynchronize(c.s));
  if (info) {
    info->iters = it;
    info->n_converged = nconv + 1;
    info->spmm_columns = c.spmm_cols;
    info->max_residual = maxres;
  }
  if (nconv < k) {
    set_error("eigensolver: %d of %d pairs above tol %.3g after %d iterations (max residual %.3g)", k - nconv, k,
              o->tol, it, maxres);
    return RW_ENOCONV;
  }
  return RW_OK;
}

static int validate_eig(const Graph* g, int m, const rw_eig_opts* o, int* nb) {
  RW_CHECK(o != nullptr, RW_EINVAL, "null options");
  RW_CHECK(o->q_dtype == g->dtype, RW_EINVAL, "Q dtype must equal the graph dtype");
  RW_CHECK(std::isfinite(o->tol) && o->tol > 0.0, RW_EINVAL, "tol must be > 0");
  RW_CHECK(m >= 2, RW_EINVAL, "m must be >= 2");
  *nb = m - 1 + guard_of(m, o);
  RW_CHECK(*nb <= g->N - 1, RW_EINVAL, "m + guard = %d exceeds N - 1 = %lld", *nb + 1, (long long)(g->N - 1));
  RW_CHECK(*nb <= 1022, RW_EINVAL, "block of %d columns exceeds the dense eigensolver limit", *nb);
  return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_eig_workspace_bytes(rw_graph h, int m, const rw_eig_opts* opts, size_t* bytes) {
  RW_CHECK(h != nullptr && bytes != nullptr, RW_EINVAL, "null argument");
  int nb = 0;
  RW_TRY(validate_eig(&h->g, m, opts, &nb));
  *bytes = eig_layout(&h->g, nb, nullptr, nullptr);
  return RW_OK;
}

int rw_precompute_eig(rw_graph h, int m, const rw_eig_opts* opts, void* Q, double* lambda, void* work,
                      size_t work_bytes, hipStream_t stream, rw_eig_info* info) {
  RW_NOT_CAPTURING(stream);
  auto t0 = std::chrono::steady_clock::now();
  RW_CHECK(h != nullptr && Q != nullptr && lambda != nullptr && work != nullptr, RW_EINVAL, "null argument");
  const Graph* g = &h->g;
  int nb = 0;
  RW_TRY(validate_eig(g, m, opts, &nb));
  Ctx c;
  c.g = g;
  c.dt = g->dtype;
  c.N = g->N;
  c.s = stream;
  c.floor_rel = g->dtype == RW_F64 ? 1e-28 : 1e-14;
  size_t need = eig_layout(g, nb, work, &c.w);
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "eig workspace too small: %zu < %zu", work_bytes, need);
  if (opts->warm) {
    RW_TRY(copy_cols(opts->q_dtype, (const char*)Q + dtype_size(opts->q_dtype) * g->N, g->N, c.dt, c.w.B[0], g->N,
                     g->N, m - 1, stream));
    RW_TRY(fill_random(c.dt, c.w.B[0] + dtype_size(c.dt) * g->N * (m - 1), g->N, g->N, nb - (m - 1), opts->seed,
                       stream));
  } else {
    RW_TRY(fill_random(c.dt, c.w.B[0], g->N, g->N, nb, opts->seed, stream));
  }
  int st = chfsi(c, m, nb, opts, Q, lambda, info);
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

int rw_update_workspace_bytes(rw_graph h, int m, const rw_eig_opts* opts, size_t* bytes) {
  return rw_eig_workspace_bytes(h, m, opts, bytes);
}

int rw_update_eig(rw_graph h, const rw_edit* edits, int n_edits, int mode, const rw_eig_opts* opts, void* Q,
                  double* lambda, int m, void* work, size_t work_bytes, hipStream_t stream, rw_eig_info* info) {
  RW_NOT_CAPTURING(stream);
  auto t0 = std::chrono::steady_clock::now();
  RW_CHECK(h != nullptr && Q != nullptr && lambda != nullptr && work != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(mode >= RW_UPDATE_DIAG_RQ && mode <= RW_UPDATE_RR_REFINE, RW_EINVAL, "unknown update mode %d", mode);
  Graph* g = &h->g;
  int nb = 0;
  RW_TRY(validate_eig(g, m, opts, &nb));
  Ctx c;
  c.g = g;
  c.dt = g->dtype;
  c.N = g->N;
  c.s = stream;
  c.floor_rel = g->dtype == RW_F64 ? 1e-28 : 1e-14;
  size_t need = eig_layout(g, nb, work, &c.w);
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "update workspace too small: %zu < %zu", work_bytes, need);
  RW_TRY(rw_edit_graph(h, edits, n_edits, stream));
  EigWork& w = c.w;
  const int k = m - 1;
  const size_t es = dtype_size(c.dt);
  // Rayleigh-Ritz on a basis stored in the graph's type reads Q's columns directly (the projection writes the
  // block) and writes the rotated basis straight back into Q
  const bool direct = mode == RW_UPDATE_RR && opts->q_dtype == c.dt;
  char* Qv = (char*)Q + dtype_size(opts->q_dtype) * g->N;   // columns 1..m-1
  if (!direct)
    RW_TRY(copy_cols(opts->q_dtype, Qv, g->N, c.dt, w.B[0], g->N, g->N, k, stream));
  int st = RW_OK;
  if (mode == RW_UPDATE_RR_REFINE) {
    RW_TRY(fill_random(c.dt, w.B[0] + es * g->N * k, g->N, g->N, nb - k, opts->seed ^ 0x5eedull, stream));
    st = chfsi(c, m, nb, opts, Q, lambda, info);
  } else {
    // Rayleigh-Ritz in place on an FP32 basis: Q's column 0 takes the edited graph's null vector and the
    // projection folds into the step (the rotation reads each row of [g, Qv] before writing it)
    const bool fold = mode == RW_UPDATE_RR && direct && c.dt == RW_F32 && k + 1 <= nb &&
                      gemm_rowwise(c.dt, c.N, k + 1, k);
    if (fold) RW_TRY(copy_cols(c.dt, g->ghat, c.N, c.dt, Q, c.N, c.N, 1, stream));
    else if (direct) RW_TRY(project_out_to(c.dt, Qv, c.N, w.B[0], c.N, g->ghat, c.N, k, w.tmp, w.partial, stream));
    else RW_TRY(project_out(c.dt, w.B[0], c.N, g->ghat, c.N, k, w.tmp, w.partial, stream));
    int ix = 0;
    if (mode == RW_UPDATE_DIAG_RQ) {
      // order-preserving orthonormalization (Cholesky QR, twice), then lambda_i = q_i^T op q_i
      int src = 0;
      for (int pass = 0; pass < 2; ++pass) {
        int dst = pass == 0 ? 1 : 2;
        RW_TRY(gram(c.dt, w.B[src], c.N, w.B[src], c.N, c.N, k, k, w.G, w.partial, stream, true));
        RW_TRY(chol_inverse(w.G, w.W, k, w.info, stream));
        int bad = 0;
        RW_HIP(hipMemcpyAsync(&bad, w.info, sizeof(int), hipMemcpyDeviceToHost, stream));
        RW_HIP(hipStreamSynchronize(stream));
        RW_CHECK(bad == 0, RW_ESINGULAR, "stored eigenvectors are linearly dependent after the edit (pivot %d)", bad);
        RW_TRY(gemm_tn(c.dt, w.B[src], c.N, w.W, k, w.B[dst], c.N, c.N, k, k, 0.0, stream));
        src = dst;
      }
      ix = 2;
      RW_TRY(stencil_apply(g, w.B[ix], w.B[3], nullptr, k, 1.0, 0.0, 0.0, stream));
      c.spmm_cols += k;
      RW_TRY(col_dots(c.dt, w.B[ix], w.B[3], c.N, k, c.N, w.theta, w.partial, stream));
      RW_TRY(residual_norms(c.dt, w.B[3], w.B[ix], w.theta, c.N, k, c.N, w.res, w.partial, stream));
    } else {
      RW_TRY(rr_step(c, k, fold ? Qv : w.B[0], w.B[1], direct ? Qv : w.B[2], w.B[3], true, fold));
      ix = 2;
    }
    const int qdt = opts->q_dtype;
    RW_TRY(copy_cols(c.dt, g->ghat, c.N, qdt, Q, c.N, c.N, 1, stream));
    if (!direct) RW_TRY(copy_cols(c.dt, w.B[ix], c.N, qdt, Qv, c.N, c.N, k, stream));
    RW_HIP(hipMemsetAsync(lambda, 0, sizeof(double), stream));   // lambda[0] = +0.0
    RW_HIP(hipMemcpyAsync(lambda + 1, w.theta, k * sizeof(double), hipMemcpyDeviceToDevice, stream));
    void* stage = nullptr;
    RW_TRY(host_stage(k * sizeof(double), &stage));
    RW_HIP(hipMemcpyAsync(stage, w.res, k * sizeof(double), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipStreamSynchronize(stream));
    const std::vector<double> rs(static_cast<double*>(stage), static_cast<double*>(stage) + k);
    if (info) {
      info->iters = 0;
      info->spmm_columns = c.spmm_cols;
      double mr = 0.0;
      int nc = 0;
      for (double r : rs) {
        mr = std::max(mr, r);
        nc += r <= opts->tol;
      }
      info->max_residual = mr;
      info->n_converged = nc + 1;
    }
  }
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

}  // extern "C"
