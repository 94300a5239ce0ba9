// Matrix-free stencil operator: Y = alpha * op(X) + beta * X + gamma * Z for a column-major N x b
// block, op = L_hat = I - D^{-1/2} W D^{-1/2} (zero rows where d = 0) or L = D - W (Sec. II-A, Sec. II-C).
//
// Per node the operator needs the diagonal and the coefficients of its 4/8/6 incident edges:
// forward edges are stored at the node, backward ones at the neighbour (the edge's tail).
//
// Main kernel (k_stencil_strip): each thread owns a strip of R nodes along y (2D: 4 in FP32, 2 in FP64) or
// z (3D: 4) at one x,
// holds their coefficients in registers, and walks its group of columns.  Per column it loads the
// strip's centre values plus one row above and below once (register window, so the strip direction's
// neighbours are not re-read), the x +- 1 values, and in 3D the y +- 1 values; the next column's
// window is loaded before the current one is computed (two windows in flight).  Y is written with
// non-temporal stores (it is not re-read by this launch).  The columns are split into G groups on
// gridDim.y so that small grids still fill the chip; tiles are dealt to the 8 XCDs in contiguous
// ranges (workgroup w runs on XCD w mod 8), so the rows a tile shares with its neighbours sit in the
// same L2.  Byte offsets within a column are 32-bit; larger grids take the plain one-node-per-thread
// kernel (k_stencil_wide).
#include <hip/hip_ext.h>

#include "rw_internal.h"

namespace rw {

template <typename T>
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

struct StripMap {
  int tiles_x;   // 64-wide tiles along x
  int tiles_y;   // 3D: 4-row tiles along y
  int ntiles;
  int per_xcd;   // tiles per XCD (gridDim.x = 8 * per_xcd)
  int cpg;       // columns per group (gridDim.y groups)
};

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// Buffer loads and stores: a resource based at a column group's first column, the column's byte offset as
// the scalar offset and the lane's 32-bit node offset as the vector offset, so no per-lane 64-bit address
// is formed (or kept across the column loop); an offset past the resource reads 0.  Stores are non-temporal.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}
template <typename T> struct Buf;
template <> struct Buf<float> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
  }
  static __device__ __forceinline__ void st(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, vo, so, 2);
  }
};
template <> struct Buf<double> {
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  }
  static __device__ __forceinline__ void st(double v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(
                                              r, vo, so, 0)), v), r, vo, so, 2);
  }
};

// ZT: the launch adds gamma Z (the fused Chebyshev step), with Z prefetched in the window like X.  alpha and
// beta are folded into the per-thread coefficients (diagonal alpha d + beta, off-diagonals alpha c), so a node
// costs the same multiply-adds in every mode; with alpha = 1 and beta = 0 the arithmetic is the plain operator's.
// Neighbour offsets are the centre offset plus per-thread deltas (0 at a clamped boundary, whose coefficient is
// 0).  BUF: buffer loads and stores (about 100 VGPRs for FP32); otherwise global loads and non-temporal stores
// through 64-bit addresses (the compiler keeps one per load, about 180 VGPRs at R = 4).  Which is faster depends
// on the mode (measured from HBM, each launch after a 1.25 GiB write and a 512 MiB read, MI355X):
//   512 x 512 8-conn FP32, 219 columns, plain:  global R = 2 109 us, buffer R = 4 115 us, buffer R = 2 118 us;
//                                       fused:  buffer R = 4 147 us, global R = 4 149 us, global R = 2 157 us;
//   128^3 6-conn FP32, 110 columns, plain:      buffer R = 4 491 us, global R = 4 498 us, R = 2 530-545 us;
//                                   fused:      buffer R = 4 638 us, global R = 4 695 us, R = 2 684-694 us;
// all with two column groups (one or four were slower).  The 3D kernel runs at the same speed from HBM as from
// the caches (about 0.48 of 8 TB/s): it is bound by its loads' issue, not by HBM.
// 2D tiles: WX waves side by side along x (64 WX columns) and 4 / WX strips along y.  For the 2D plain operator
// (the eigensolver's residual and Rayleigh-Ritz products) tiles two waves wide with 8-row strips, buffer loads
// and four column groups took 95 us against 110 us for the 64-wide tiles (copy of the same bytes: 81 us;
// 8-wide strips of one-wave tiles, R = 4 or 16, or eight groups were slower; taking x +- 1 from neighbouring
// lanes by DPP wave shifts instead of loads took 143 us).  AB: alpha and beta are folded into the coefficients
// (off for the plain operator, which then uses them as stored; with the folding the same tiles took 114 us).
// PF: columns in flight ahead of the one computed (1 or 2).  For the 2D plain tiles, two took 97-98 us against
// 100-103 us for one (eight column groups: 105-110 us; R = 4 with eight groups: 100-101 us); back to back
// 77 us either way, so the remaining distance to the copy is the latency of the first loads from HBM.
template <typename T, int NDIR, int R, bool ZT, bool BUF, int WX = 1, bool AB = true, int PF = 1>
__global__ __launch_bounds__(256) void k_stencil_strip(StencilArgs<T> a, StripMap tm) {
  using C = typename Elem<T>::C;
  constexpr bool D3 = NDIR == 3;
  constexpr bool DIAG = NDIR == 4;
  const int bid = blockIdx.x;
  const int tile = (bid & 7) * tm.per_xcd + (bid >> 3);
  if (tile >= tm.ntiles) return;
  const int nx = (int)a.G.nx, ny = (int)a.G.ny, nz = (int)a.G.nz, N = (int)a.G.N;
  const int tx = tile % tm.tiles_x;
  const int t2 = tile / tm.tiles_x;
  static_assert(WX == 1 || !D3, "3D tiles are one wave wide");
  const int x = (tx * WX + (int)threadIdx.y % WX) * 64 + threadIdx.x;
  int y = 0, s0 = 0;     // 3D: y row and first z of the strip; 2D: first y of the strip
  if constexpr (D3) {
    y = (t2 % tm.tiles_y) * 4 + threadIdx.y;
    s0 = (t2 / tm.tiles_y) * R;
    if (x >= nx || y >= ny) return;
  } else {
    s0 = (t2 * (4 / WX) + (int)threadIdx.y / WX) * R;
    if (x >= nx || s0 >= ny) return;
  }
  const int plane = nx * ny;
  // window rows p = 0..R+1 are strip positions s0 - 1 .. s0 + R (clamped; their coefficients are 0)
  uint32_t oc[R + 2];
#pragma unroll
  for (int p = 0; p < R + 2; ++p) {
    const int row = D3 ? nx * y + plane * clampi(s0 + p - 1, nz) : nx * clampi(s0 + p - 1, ny);
    oc[p] = (uint32_t)(x + row) * (uint32_t)sizeof(T);
  }
  const uint32_t es = (uint32_t)sizeof(T);
  const uint32_t dl = x > 0 ? es : 0u, dr = x + 1 < nx ? es : 0u;   // x - 1 = oc - dl, x + 1 = oc + dr
  uint32_t dyp = 0, dym = 0;                                        // 3D: y +- 1
  if constexpr (D3) {
    dyp = y + 1 < ny ? (uint32_t)nx * es : 0u;
    dym = y > 0 ? (uint32_t)nx * es : 0u;
  }
  const C al = a.alpha, be = a.beta, ga = a.gamma;
  C c[R][2 * NDIR];
  C dg[R];
  bool ok[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    int yy, zz;
    if constexpr (D3) {
      yy = y;
      zz = s0 + k;
      ok[k] = zz < nz;
      zz = clampi(zz, nz);
    } else {
      yy = s0 + k;
      zz = 0;
      ok[k] = yy < ny;
      yy = clampi(yy, ny);
    }
    const int i = x + nx * yy + plane * zz;
    dg[k] = ok[k] ? (AB ? al * (C)a.diag[i] + be : (C)a.diag[i]) : C(0);
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
      const int hx = x + a.G.dx[d], hy = yy + a.G.dy[d], hz = zz + a.G.dz[d];
      const bool f = ok[k] && hx >= 0 && hx < nx && hy >= 0 && hy < ny && hz >= 0 && hz < nz;
      c[k][d] = f ? (AB ? al : C(1)) * (C)a.coef[d * N + i] : C(0);
      const int ux = x - a.G.dx[d], uy = yy - a.G.dy[d], uz = zz - a.G.dz[d];
      const bool t = ok[k] && ux >= 0 && ux < nx && uy >= 0 && uy < ny && uz >= 0 && uz < nz;
      c[k][NDIR + d] = t ? (AB ? al : C(1)) * (C)a.coef[d * N + i - (int)a.G.off[d]] : C(0);
    }
  }
  const int c0 = blockIdx.y * tm.cpg;
  const int c1 = (int)min((int64_t)c0 + tm.cpg, a.b);
  if (c0 >= c1) return;
  const size_t cs = (size_t)N * sizeof(T);   // the host keeps (cpg - 1) cs + cs below 2^32
  const __amdgpu_buffer_rsrc_t rx = buf_rsrc(reinterpret_cast<const char*>(a.X) + (size_t)c0 * cs);
  const __amdgpu_buffer_rsrc_t ry = buf_rsrc(reinterpret_cast<const char*>(a.Y) + (size_t)c0 * cs);
  const __amdgpu_buffer_rsrc_t rz = buf_rsrc(ZT ? reinterpret_cast<const char*>(a.Z) + (size_t)c0 * cs
                                                : reinterpret_cast<const char*>(a.X));
  struct Win {
    C cen[R + 2], lf[R + 2], rt[R + 2];
    C yp[D3 ? R : 1], ym[D3 ? R : 1];
    C z[ZT ? R : 1];
  };
  const char* xg = reinterpret_cast<const char*>(a.X) + (size_t)c0 * cs;
  const char* zg = ZT ? reinterpret_cast<const char*>(a.Z) + (size_t)c0 * cs : xg;
  char* yg = reinterpret_cast<char*>(a.Y) + (size_t)c0 * cs;
  auto ldx = [&](uint32_t so, uint32_t o) -> C {
    if constexpr (BUF) return (C)Buf<T>::ld(rx, o, so);
    else return (C)*reinterpret_cast<const T*>(xg + so + o);
  };
  auto ldz = [&](uint32_t so, uint32_t o) -> C {
    if constexpr (BUF) return (C)Buf<T>::ld(rz, o, so);
    else return (C)*reinterpret_cast<const T*>(zg + so + o);
  };
  auto load = [&](Win& w, uint32_t so) {
#pragma unroll
    for (int q = 0; q < R + 2; ++q) {
      w.cen[q] = ldx(so, oc[q]);
      if (DIAG || (q >= 1 && q <= R)) {
        w.lf[q] = ldx(so, oc[q] - dl);
        w.rt[q] = ldx(so, oc[q] + dr);
      } else {
        w.lf[q] = C(0);
        w.rt[q] = C(0);
      }
    }
    if constexpr (D3) {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        w.yp[k] = ldx(so, oc[k + 1] + dyp);
        w.ym[k] = ldx(so, oc[k + 1] - dym);
      }
    }
    if constexpr (ZT) {
#pragma unroll
      for (int k = 0; k < R; ++k) w.z[k] = ldz(so, oc[k + 1]);
    }
  };
  auto compute = [&](const Win& w, uint32_t so) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int p = k + 1;
      C acc = dg[k] * w.cen[p];
      // heads d = 0..NDIR-1, then tails (the edge order the graph defines)
      if constexpr (NDIR == 2) {
        acc -= c[k][0] * w.rt[p];
        acc -= c[k][1] * w.cen[p + 1];
        acc -= c[k][2] * w.lf[p];
        acc -= c[k][3] * w.cen[p - 1];
      } else if constexpr (NDIR == 4) {
        acc -= c[k][0] * w.rt[p];
        acc -= c[k][1] * w.cen[p + 1];
        acc -= c[k][2] * w.rt[p + 1];
        acc -= c[k][3] * w.rt[p - 1];
        acc -= c[k][4] * w.lf[p];
        acc -= c[k][5] * w.cen[p - 1];
        acc -= c[k][6] * w.lf[p - 1];
        acc -= c[k][7] * w.lf[p + 1];
      } else {
        acc -= c[k][0] * w.rt[p];
        acc -= c[k][1] * w.yp[k];
        acc -= c[k][2] * w.cen[p + 1];
        acc -= c[k][3] * w.lf[p];
        acc -= c[k][4] * w.ym[k];
        acc -= c[k][5] * w.cen[p - 1];
      }
      if constexpr (ZT) acc += ga * w.z[k];
      if (ok[k]) {
        if constexpr (BUF) Buf<T>::st((T)acc, ry, oc[p], so);
        else __builtin_nontemporal_store((T)acc, reinterpret_cast<T*>(yg + so + oc[p]));
      }
    }
  };
  const uint32_t ucs = (uint32_t)cs;
  uint32_t so = 0;
  int col = c0;
  if constexpr (PF == 1) {   // one column in flight ahead of the one computed
    Win w0, w1;
    load(w0, 0u);
    for (; col + 2 <= c1; col += 2) {
      load(w1, so + ucs);
      compute(w0, so);
      if (col + 2 < c1) load(w0, so + 2 * ucs);
      compute(w1, so + ucs);
      so += 2 * ucs;
    }
    if (col < c1) compute(w0, so);
  } else {                   // two columns in flight: three windows in rotation
    Win w0, w1, w2;
    load(w0, 0u);
    if (col + 1 < c1) load(w1, ucs);
    for (; col + 3 <= c1; col += 3) {
      load(w2, so + 2 * ucs);
      compute(w0, so);
      if (col + 3 < c1) load(w0, so + 3 * ucs);
      compute(w1, so + ucs);
      if (col + 4 < c1) load(w1, so + 4 * ucs);
      compute(w2, so + 2 * ucs);
      so += 3 * ucs;
    }
    if (col < c1) compute(w0, so);
    if (col + 1 < c1) compute(w1, so + ucs);
  }
}

// one node per thread, all columns, 64-bit indexing (grids whose columns exceed 32-bit byte offsets)
template <typename T, int NDIR>
__global__ __launch_bounds__(256) void k_stencil_wide(StencilArgs<T> a) {
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

// Strip length and column groups.  Groups: enough threads to cover the chip about once (256 CUs x 1024
// threads), at least 4 columns per group, at most 8 groups; gforce > 0 fixes the number of groups (still
// doubled while the 32-bit offsets need it).  WX: waves per tile along x (2D).
template <int NDIR>
static StripMap strip_map(const Graph* g, int R, int64_t b, dim3* grid, int WX = 1, int gforce = 0) {
  StripMap tm;
  tm.tiles_x = (int)nblocks(g->nx, 64 * WX);
  int64_t strips;
  if (NDIR == 3) {
    tm.tiles_y = (int)nblocks(g->ny, 4);
    strips = (int64_t)tm.tiles_x * tm.tiles_y * nblocks(g->nz, R);
    tm.ntiles = (int)strips;
  } else {
    tm.tiles_y = 0;
    tm.ntiles = (int)((int64_t)tm.tiles_x * nblocks(nblocks(g->ny, R), 4 / WX));
  }
  const int64_t threads = (int64_t)tm.ntiles * 256;
  int G = 1;
  while (G < 8 && threads * G < (int64_t)256 * 1024 && (b + 2 * G - 1) / (2 * G) >= 4) G *= 2;
  if (threads >= 64 * 1024 && b >= 8) G = 2;   // large grids: two groups (measured best, see the kernel)
  if (gforce > 0) G = (int)std::max<int64_t>(1, std::min<int64_t>(gforce, b));
  tm.cpg = (int)((b + G - 1) / G);
  // the buffer offsets of a column group, (cpg - 1) cs + node offsets, stay below 2^32
  const uint64_t cs = (uint64_t)g->N * dtype_size(g->dtype);
  while ((uint64_t)tm.cpg * cs >= ((uint64_t)1 << 32)) {
    G *= 2;
    tm.cpg = (int)((b + G - 1) / G);
  }
  tm.per_xcd = (tm.ntiles + 7) / 8;
  *grid = dim3((unsigned)(tm.per_xcd * 8), (unsigned)G);
  return tm;
}

// a kernel launch; with events, through hipExtLaunchKernel so that they record this dispatch's own start
// and end (the interval a kernel trace reports), not the stream's progress around it
template <typename... A>
static hipError_t launch_k(void (*kernel)(A...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1, A... args) {
  if (e0 == nullptr && e1 == nullptr) {
    kernel<<<grid, block, 0, s>>>(args...);
    return hipGetLastError();
  }
  void* argv[] = {static_cast<void*>(&args)...};
  return hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, argv, 0, s, e0, e1, 0);
}

template <typename T, int NDIR>
static int launch(const Graph* g, const void* X, void* Y, const void* Z, int64_t b, double alpha,
                  double beta, double gamma, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  using C = typename Elem<T>::C;
  StencilArgs<T> a;
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
  hipError_t st = hipSuccess;
  const bool narrow = (uint64_t)g->N * sizeof(T) < ((uint64_t)1 << 31) && b < (int64_t)1 << 30;
  if (narrow) {
    dim3 grid;
    const bool zt = a.Z != nullptr;
    if constexpr (NDIR == 3) {                       // 3D: buffer loads, four nodes per thread along z
      StripMap tm = strip_map<NDIR>(g, 4, b, &grid);
      if (zt) st = launch_k(k_stencil_strip<T, NDIR, 4, true, true>, grid, block, s, e0, e1, a, tm);
      else st = launch_k(k_stencil_strip<T, NDIR, 4, false, true>, grid, block, s, e0, e1, a, tm);
    } else if (zt && sizeof(T) == 4) {               // 2D fused FP32: buffer loads, four nodes per thread
      StripMap tm = strip_map<NDIR>(g, 4, b, &grid);
      st = launch_k(k_stencil_strip<T, NDIR, 4, true, true>, grid, block, s, e0, e1, a, tm);
    } else if (sizeof(T) == 4 && alpha == 1.0 && beta == 0.0) {
      // 2D plain FP32: 128-column tiles of two 8-row strips, buffer loads, four column groups, two columns
      // in flight
      StripMap tm = strip_map<NDIR>(g, 8, b, &grid, 2, 4);
      st = launch_k(k_stencil_strip<T, NDIR, 8, false, true, 2, false, 2>, grid, block, s, e0, e1, a, tm);
    } else {                                         // 2D plain, and FP64: global loads, two nodes per thread
      StripMap tm = strip_map<NDIR>(g, 2, b, &grid);
      if (zt) st = launch_k(k_stencil_strip<T, NDIR, 2, true, false>, grid, block, s, e0, e1, a, tm);
      else st = launch_k(k_stencil_strip<T, NDIR, 2, false, false>, grid, block, s, e0, e1, a, tm);
    }
  } else {
    RW_CHECK(g->ny * g->nz < (int64_t)4 * 65535, RW_EINVAL, "grid too tall for the stencil launch");
    dim3 grid(nblocks(g->nx, 64), nblocks(g->ny * g->nz, 4));
    st = launch_k(k_stencil_wide<T, NDIR>, grid, block, s, e0, e1, a);
  }
  RW_CHECK(st == hipSuccess, RW_EHIP, "stencil launch: %s", hipGetErrorString(st));
  return RW_OK;
}

int stencil_apply(const Graph* g, const void* X, void* Y, const void* Z, int64_t b, double alpha,
                  double beta, double gamma, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (b <= 0) return RW_OK;
  if (g->dtype == RW_F64) {
    switch (g->ndir) {
      case 2: return launch<double, 2>(g, X, Y, Z, b, alpha, beta, gamma, s, e0, e1);
      case 3: return launch<double, 3>(g, X, Y, Z, b, alpha, beta, gamma, s, e0, e1);
      default: return launch<double, 4>(g, X, Y, Z, b, alpha, beta, gamma, s, e0, e1);
    }
  }
  switch (g->ndir) {
    case 2: return launch<float, 2>(g, X, Y, Z, b, alpha, beta, gamma, s, e0, e1);
    case 3: return launch<float, 3>(g, X, Y, Z, b, alpha, beta, gamma, s, e0, e1);
    default: return launch<float, 4>(g, X, Y, Z, b, alpha, beta, gamma, s, e0, e1);
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

int rw_apply_laplacian_timed(rw_graph h, const void* X, void* Y, int64_t b, hipStream_t stream,
                             hipEvent_t start, hipEvent_t stop) {
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  RW_CHECK(b >= 1, RW_EINVAL, "b must be >= 1");
  RW_CHECK(X != nullptr && Y != nullptr, RW_EINVAL, "null X or Y");
  RW_CHECK(X != Y, RW_EINVAL, "X and Y must be distinct");
  RW_CHECK(start != nullptr && stop != nullptr, RW_EINVAL, "null event");
  return stencil_apply(&h->g, X, Y, nullptr, b, 1.0, 0.0, 0.0, stream, start, stop);
}

}  // extern "C"
