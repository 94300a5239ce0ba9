// Image graph: edge weights, degrees, null vector and stencil coefficients (Sec. II-A eq. (2),
// Sec. II-C), and graph edits (Sec. III-B and weight / topology edits).
#include <cmath>
#include <cstdarg>
#include <algorithm>
#include <cstring>
#include <vector>

#include "rw_internal.h"

namespace rw {

static thread_local char g_last_error[1024];   // fixed storage: reporting an error allocates nothing

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}

static thread_local void* g_stage = nullptr;
static thread_local size_t g_stage_cap = 0;

int host_stage(size_t bytes, void** p) {
  if (g_stage_cap < bytes) {
    if (g_stage != nullptr) RW_HIP(hipHostFree(g_stage));
    g_stage = nullptr;
    g_stage_cap = 0;
    const size_t cap = std::max<size_t>(bytes, 65536);
    RW_HIP(hipHostMalloc(&g_stage, cap, hipHostMallocDefault));
    g_stage_cap = cap;
  }
  *p = g_stage;
  return RW_OK;
}

static constexpr int64_t kEditStage = 65536;  // edge ids staged per chunk of an edit list

__global__ void k_graph_init(GridDev G, const void* Jsrc, int Jdt, double* J, double* scale, uint8_t* mask) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  J[i] = Jdt == RW_F64 ? static_cast<const double*>(Jsrc)[i] : (double)static_cast<const float*>(Jsrc)[i];
  int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / (G.nx * G.ny);
  uint8_t m = 0;
  for (int d = 0; d < G.ndir; ++d) {
    bool ok = head_in(G, x, y, z, d);
    scale[d * G.N + i] = ok ? 1.0 : 0.0;
    if (ok) m |= uint8_t(1u << d);
  }
  mask[i] = m;
}

// w_e = s_e * exp(-beta * f(J_tail - J_head)) in FP64.  Scales, weights and degrees are FP64 on every
// graph; only the operator's coefficients (coef, diag, dinv, ghat) take the graph's type, so the seed
// rows of the online solve can be formed from FP64 values on an FP32 graph.
// `flip` is set when an edge's weight crosses kAnchorWeight (the connectivity used by the solvability
// check changes only then); it reads the previous weights, so on a first build it means nothing.
__global__ void k_weights(GridDev G, const double* J, double beta, int form, const double* scale,
                          const uint8_t* mask, double* weight, int* flip) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  uint8_t m = mask[i];
  bool crossed = false;
  for (int d = 0; d < G.ndir; ++d) {
    double w = 0.0;
    if ((m >> d) & 1u) {
      double diff = J[i] - J[i + G.off[d]];
      double e = form == RW_WEIGHT_SQUARED ? diff * diff : fabs(diff);
      w = scale[d * G.N + i] * exp(-beta * e);
    }
    const double old = weight[d * G.N + i];
    crossed |= (old >= kAnchorWeight) != (w >= kAnchorWeight);
    weight[d * G.N + i] = w;
  }
  if (crossed) *flip = 1;
}

// degree: forward edges stored at i, backward edges stored at the tail i - off[d]; fixed order.
__global__ void k_degree(GridDev G, const double* weight, double* degree, double* partial) {
  double local = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G.N;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / (G.nx * G.ny);
    double d = 0.0;
    for (int k = 0; k < G.ndir; ++k) d += weight[k * G.N + i];
    for (int k = 0; k < G.ndir; ++k)
      if (tail_in(G, x, y, z, k)) d += weight[k * G.N + i - G.off[k]];
    degree[i] = d;
    local += d;
  }
  // block reduction in fixed order
  __shared__ double sh[256];
  sh[threadIdx.x] = local;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_sum_partials(const double* partial, int n, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

template <typename T>
__global__ void k_finish(GridDev G, int normalized, const double* degree, const double* sums,
                         const double* weight, const uint8_t* mask, T* dinv, T* ghat, T* diag, T* coef) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  double d = degree[i];
  double di = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  dinv[i] = T(di);
  if (normalized) {
    ghat[i] = T(sqrt(d) / sqrt(sums[0]));
    diag[i] = T(d > 0.0 ? 1.0 : 0.0);
  } else {
    ghat[i] = T(1.0 / sqrt((double)G.N));
    diag[i] = T(d);
  }
  uint8_t m = mask[i];
  for (int k = 0; k < G.ndir; ++k) {
    double c = 0.0;
    if ((m >> k) & 1u) {
      double w = weight[k * G.N + i];
      if (normalized) {
        double dh = degree[i + G.off[k]];
        double dhi = dh > 0.0 ? 1.0 / sqrt(dh) : 0.0;
        c = w * di * dhi;
      } else {
        c = w;
      }
    }
    coef[k * G.N + i] = T(c);
  }
}

__global__ void k_scale_box(GridDev G, int64_t x0, int64_t y0, int64_t z0, int64_t x1, int64_t y1,
                            int64_t z1, double v, const uint8_t* mask, double* scale) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / (G.nx * G.ny);
  if (x < x0 || x >= x1 || y < y0 || y >= y1 || z < z0 || z >= z1) return;
  uint8_t m = mask[i];
  for (int d = 0; d < G.ndir; ++d) {
    if (!((m >> d) & 1u)) continue;
    int64_t a = x + G.dx[d], b = y + G.dy[d], c = z + G.dz[d];
    if (a < x0 || a >= x1 || b < y0 || b >= y1 || c < z0 || c >= z1) continue;
    scale[d * G.N + i] *= v;
  }
}

// ids are distinct within one launch (checked on the host), so no two threads touch one slot.
__global__ void k_edit_ids(const int64_t* ids, int64_t n, double v, int remove, double* scale) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  int64_t e = ids[k];
  scale[e] = remove ? 0.0 : scale[e] * v;
}

size_t graph_layout(const rw_graph_desc& d, Graph* g, void* buf) {
  int64_t N = d.dims[0] * d.dims[1] * d.dims[2];
  int nd = d.ndim == 3 ? 3 : (d.conn == 8 ? 4 : 2);
  size_t es = dtype_size(d.dtype);
  Carver c(buf);
  double* J = c.take<double>(N);
  double* scale = c.take<double>(nd * N);
  double* weight = c.take<double>(nd * N);
  char* coef = c.take<char>(nd * N * es);
  char* diag = c.take<char>(N * es);
  char* dinv = c.take<char>(N * es);
  char* ghat = c.take<char>(N * es);
  double* degree = c.take<double>(N);
  uint8_t* mask = c.take<uint8_t>(N);
  double* partial = c.take<double>(kReduceBlocks);
  double* sums = c.take<double>(8);
  int64_t* comp = c.take<int64_t>(N);
  int* ccf = c.take<int>(64);
  c.take<int64_t>(kEditStage);       // must stay the last block (edit_stage)
  if (g) {
    g->J = J; g->scale = scale; g->weight = weight; g->coef = coef; g->diag = diag; g->dinv = dinv;
    g->ghat = ghat; g->degree = degree; g->mask = mask; g->partial = partial; g->sums = sums;
    g->comp = comp; g->cc_flag = ccf; g->cc_valid = false;
  }
  return c.used;
}

static int64_t* edit_stage(const Graph* g) {
  // the staging area is the last block of the layout: recompute its offset
  rw_graph_desc d{};
  d.ndim = g->ndim; d.dims[0] = g->nx; d.dims[1] = g->ny; d.dims[2] = g->nz; d.conn = g->conn;
  d.dtype = g->dtype;
  size_t total = graph_layout(d, nullptr, nullptr);
  size_t off = total - kEditStage * sizeof(int64_t);
  return reinterpret_cast<int64_t*>(reinterpret_cast<char*>(g->J) + off);
}

template <typename T>
static int rebuild_t(Graph* g, hipStream_t s) {
  GridDev G = grid_of(g);
  const int t = 256;
  k_weights<<<nblocks(g->N, t), t, 0, s>>>(G, g->J, g->beta, g->weight_form, g->scale, g->mask, g->weight,
                                             g->cc_flag + 4);
  RW_LAUNCH_CHECK();
  int nb = (int)std::min<int64_t>(kReduceBlocks, nblocks(g->N, t));
  k_degree<<<nb, t, 0, s>>>(G, g->weight, g->degree, g->partial);
  RW_LAUNCH_CHECK();
  k_sum_partials<<<1, 256, 0, s>>>(g->partial, nb, g->sums);
  RW_LAUNCH_CHECK();
  k_finish<T><<<nblocks(g->N, t), t, 0, s>>>(G, g->normalized, g->degree, g->sums, g->weight,
                                               g->mask, (T*)g->dinv, (T*)g->ghat, (T*)g->diag, (T*)g->coef);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

int graph_rebuild(Graph* g, hipStream_t s) {
  if (g->cc_valid) {   // start watching for anchoring edges that appear or vanish
    RW_HIP(hipMemsetAsync(g->cc_flag + 4, 0, sizeof(int), s));
    g->cc_recheck = true;
  }
  g->cc_valid = false;
  return g->dtype == RW_F64 ? rebuild_t<double>(g, s) : rebuild_t<float>(g, s);
}

// ---------------------------------------------------------------------------------------------
// Connected components by hooking and pointer jumping.  comp[i] points to a smaller node of the same
// component, or to itself at a root.  A round hooks, for every edge above the anchor weight whose
// endpoints have different roots, the larger root under the smaller one (atomic minimum), then
// shortcuts every node to its root.  Rounds repeat until one finds no edge between different roots;
// the root of each component is then its smallest node index.
// ---------------------------------------------------------------------------------------------
// root of x with path halving (each visited node is re-pointed to its grandparent; pointers only move
// towards smaller indices, so concurrent halving and hooking keep every chain ending at a root)
__device__ __forceinline__ int64_t cc_find(int64_t* comp, int64_t x) {
  int64_t p = comp[x];
  while (p != x) {
    const int64_t gp = comp[p];
    if (gp != p) comp[x] = gp;
    x = p;
    p = gp;
  }
  return x;
}

// start from the smallest index among each node and its anchored forward neighbours' tails, so the
// first hooking round already sees short chains
__global__ void k_cc_init(GridDev G, const double* weight, const uint8_t* mask, int64_t* comp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  int64_t c = i;
  const int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / (G.nx * G.ny);
  for (int d = 0; d < G.ndir; ++d) {
    if (!tail_in(G, x, y, z, d)) continue;
    const int64_t t = i - G.off[d];
    if (((mask[t] >> d) & 1) && weight[d * G.N + t] >= kAnchorWeight && t < c) c = t;
  }
  comp[i] = c;
}

// 2D grids: the components within each 32 x 32 tile first, by min-label propagation over the tile's
// anchoring edges in LDS (each step also jumps through the current label, which is a node of the same
// component with an index no larger), until no label changes; then every node points to the smallest node
// of its tile-local component.  The hooking rounds then only join tiles.
__global__ __launch_bounds__(1024) void k_cc_init_tile(GridDev G, const double* weight, const uint8_t* mask,
                                                       int64_t* comp) {
  __shared__ int lab[1024];
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5, me = threadIdx.x;
  const int64_t x = (int64_t)blockIdx.x * 32 + lx, y = (int64_t)blockIdx.y * 32 + ly;
  const bool in = x < G.nx && y < G.ny;
  const int64_t i = y * G.nx + x;
  // neighbours through anchoring edges inside the tile: slot 2 d forward, 2 d + 1 backward (the node itself
  // when there is none, which changes nothing)
  int nb[8];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    nb[2 * d] = me;
    nb[2 * d + 1] = me;
    if (!in || d >= G.ndir) continue;
    if (((mask[i] >> d) & 1) && weight[d * G.N + i] >= kAnchorWeight) {   // i -> i + off[d], stored at i
      const int ax = lx + G.dx[d], ay = ly + G.dy[d];
      if (ax >= 0 && ax < 32 && ay >= 0 && ay < 32 && head_in(G, x, y, 0, d)) nb[2 * d] = ay * 32 + ax;
    }
    if (tail_in(G, x, y, 0, d)) {   // i - off[d] -> i, stored at the tail
      const int64_t t = i - G.off[d];
      const int bx = lx - G.dx[d], by = ly - G.dy[d];
      if (bx >= 0 && bx < 32 && by >= 0 && by < 32 && ((mask[t] >> d) & 1) &&
          weight[d * G.N + t] >= kAnchorWeight)
        nb[2 * d + 1] = by * 32 + bx;
    }
  }
  lab[me] = me;
  __syncthreads();
  for (;;) {
    const int cur = lab[me];
    int l = lab[cur];
#pragma unroll
    for (int c = 0; c < 8; ++c) l = min(l, lab[nb[c]]);
    const bool changed = l < cur;
    if (changed) lab[me] = l;   // labels only decrease; a concurrent reader sees either value
    if (!__syncthreads_or(changed)) break;
  }
  if (in) {
    const int r = lab[me];
    comp[i] = ((int64_t)blockIdx.y * 32 + (r >> 5)) * G.nx + (int64_t)blockIdx.x * 32 + (r & 31);
  }
}

__global__ void k_cc_hook(GridDev G, const double* weight, const uint8_t* mask, int64_t* comp, int* changed) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool valid = i < G.N;
  const uint8_t mk = valid ? mask[i] : 0;
  const int lane = threadIdx.x & 63;
  bool joined = false;
  for (int d = 0; d < G.ndir; ++d) {   // uniform: every lane reaches the shuffles
    int64_t lo = -1, hi = -1;
    if (((mk >> d) & 1) && weight[d * G.N + i] >= kAnchorWeight) {
      const int64_t a = cc_find(comp, i), b = cc_find(comp, i + G.off[d]);
      if (a != b) {
        lo = a < b ? a : b;
        hi = a < b ? b : a;
      }
    }
    // neighbouring nodes across a tile boundary mostly join the same two roots: a lane whose previous lane
    // performs the same hook leaves it to that lane (the minimum is idempotent)
    const int64_t phi = __shfl_up(hi, 1), plo = __shfl_up(lo, 1);
    if (hi >= 0 && !(lane > 0 && phi == hi && plo == lo))
      atomicMin(reinterpret_cast<unsigned long long*>(&comp[hi]), (unsigned long long)lo);
    joined = joined || hi >= 0;
  }
  // another round whenever an edge joined two roots (a concurrent hook may have re-pointed `hi` first, and
  // only a later round sees the two trees again); one store per wave, not one per join
  if (__ballot(joined) != 0 && lane == 0) *changed = 1;
}

// full compression: every node to its root.  The walk is read-only (no halving), so the only store to
// comp[i] is this thread's, and after the last round every entry is its root (the anchoring check and
// the component count rely on that).
__global__ void k_cc_jump(int64_t* comp, int64_t N) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t x = i, p = comp[i];
  while (p != x) {
    x = p;
    p = comp[x];
  }
  comp[i] = x;
}

int graph_components(Graph* g, hipStream_t s) {
  if (g->cc_valid) return RW_OK;
  if (g->cc_recheck) {   // the components of the last computation stand unless an edge crossed the threshold
    g->cc_recheck = false;
    int flip = 1;
    RW_HIP(hipMemcpyAsync(&flip, g->cc_flag + 4, sizeof(int), hipMemcpyDeviceToHost, s));
    RW_HIP(hipStreamSynchronize(s));
    if (!flip) {
      g->cc_valid = true;
      return RW_OK;
    }
  }
  const GridDev G = grid_of(g);
  if (g->nz == 1) {
    const dim3 tiles((unsigned)((g->nx + 31) / 32), (unsigned)((g->ny + 31) / 32));
    k_cc_init_tile<<<tiles, 1024, 0, s>>>(G, g->weight, g->mask, g->comp);
  } else {
    k_cc_init<<<nblocks(g->N, 256), 256, 0, s>>>(G, g->weight, g->mask, g->comp);
  }
  RW_LAUNCH_CHECK();
  auto cc_round = [&]() -> int {   // hook and jump, cc_flag[0] set when a label changed
    RW_HIP(hipMemsetAsync(g->cc_flag, 0, sizeof(int), s));
    k_cc_hook<<<nblocks(g->N, 256), 256, 0, s>>>(G, g->weight, g->mask, g->comp, g->cc_flag);
    RW_LAUNCH_CHECK();
    k_cc_jump<<<nblocks(g->N, 256), 256, 0, s>>>(g->comp, g->N);
    RW_LAUNCH_CHECK();
    return RW_OK;
  };
  // the first round's flag is not read (a round without change leaves the labels as they are, so the next
  // round reports no change either): labels are final after the first round that changes nothing
  RW_TRY(cc_round());
  for (int round = 1;; ++round) {
    RW_CHECK(round < 4096, RW_ENOCONV, "connected components did not settle");
    RW_TRY(cc_round());
    int changed = 0;
    RW_HIP(hipMemcpyAsync(&changed, g->cc_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    RW_HIP(hipStreamSynchronize(s));
    if (!changed) break;
  }
  g->cc_valid = true;
  return RW_OK;
}

__global__ void k_cc_count(const int64_t* comp, int64_t N, unsigned long long* count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N && comp[i] == i) atomicAdd(count, 1ull);
}

__global__ void k_anchor_mark(const int64_t* comp, const int64_t* seeds, int64_t S, uint8_t* flags) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < S) flags[comp[seeds[k]]] = 1;
}

__global__ void k_anchor_check(const int64_t* comp, const uint8_t* flags, int64_t N, int* bad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N && !flags[comp[i]]) *bad = 1;
}

int anchor_launch(Graph* g, const int64_t* seeds, int64_t S, uint8_t* flags, hipStream_t s, const int** bad_dev) {
  RW_TRY(graph_components(g, s));
  RW_HIP(hipMemsetAsync(flags, 0, g->N, s));
  RW_HIP(hipMemsetAsync(g->cc_flag + 1, 0, sizeof(int), s));
  k_anchor_mark<<<nblocks(std::max<int64_t>(S, 1), 256), 256, 0, s>>>(g->comp, seeds, S, flags);
  RW_LAUNCH_CHECK();
  k_anchor_check<<<nblocks(g->N, 256), 256, 0, s>>>(g->comp, flags, g->N, g->cc_flag + 1);
  RW_LAUNCH_CHECK();
  *bad_dev = g->cc_flag + 1;
  return RW_OK;
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i32(int* p, int64_t n, int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
int fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s) {
  if (n <= 0) return RW_OK;
  k_fill_u8<<<(unsigned)std::min<int64_t>(nblocks(n, 256), 4096), 256, 0, s>>>(p, n, v);
  RW_LAUNCH_CHECK();
  return RW_OK;
}
int fill_i32(int* p, int64_t n, int v, hipStream_t s) {
  if (n <= 0) return RW_OK;
  k_fill_i32<<<(unsigned)std::min<int64_t>(nblocks(n, 256), 4096), 256, 0, s>>>(p, n, v);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

int anchor_launch_async(const Graph* g, const int64_t* seeds, int64_t S, uint8_t* flags, int* bad_dev, hipStream_t s) {
  RW_CHECK(g->cc_valid, RW_EINVAL,
           "the graph's components are not current: call rw_graph_components after the last build or edit");
  RW_TRY(fill_u8(flags, g->N, 0, s));
  RW_TRY(fill_i32(bad_dev, 1, 0, s));
  k_anchor_mark<<<nblocks(std::max<int64_t>(S, 1), 256), 256, 0, s>>>(g->comp, seeds, S, flags);
  RW_LAUNCH_CHECK();
  k_anchor_check<<<nblocks(g->N, 256), 256, 0, s>>>(g->comp, flags, g->N, bad_dev);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

int check_anchored(Graph* g, const int64_t* seeds, int64_t S, uint8_t* flags, hipStream_t s) {
  const int* bad_dev = nullptr;
  RW_TRY(anchor_launch(g, seeds, S, flags, s, &bad_dev));
  int bad = 0;
  RW_HIP(hipMemcpyAsync(&bad, bad_dev, sizeof(int), hipMemcpyDeviceToHost, s));
  RW_HIP(hipStreamSynchronize(s));
  RW_CHECK(!bad, RW_EUNANCHORED,
           "a connected component (edges with w >= 1e-30) holds no seed: the gamma = 0 system is singular");
  return RW_OK;
}

static int validate_desc(const rw_graph_desc* d) {
  RW_CHECK(d != nullptr, RW_EINVAL, "null graph description");
  RW_CHECK(d->ndim == 2 || d->ndim == 3, RW_EINVAL, "ndim must be 2 or 3 (got %d)", d->ndim);
  RW_CHECK(d->dims[0] >= 1 && d->dims[1] >= 1 && d->dims[2] >= 1, RW_EINVAL, "dims must be >= 1");
  RW_CHECK(d->ndim == 3 || d->dims[2] == 1, RW_EINVAL, "a 2D graph needs dims[2] == 1");
  RW_CHECK(d->ndim == 2 ? (d->conn == 4 || d->conn == 8) : d->conn == 6, RW_EINVAL,
           "connectivity %d is not valid for %dD", d->conn, d->ndim);
  RW_CHECK(d->dtype == RW_F64 || d->dtype == RW_F32, RW_EINVAL, "graph dtype must be F64 or F32");
  RW_CHECK(d->weight_form == RW_WEIGHT_SQUARED || d->weight_form == RW_WEIGHT_ABS, RW_EINVAL,
           "unknown weight form %d", d->weight_form);
  int64_t N = d->dims[0] * d->dims[1] * d->dims[2];
  RW_CHECK(N >= 2 && N < (int64_t(1) << 40), RW_EINVAL, "N = %lld out of range", (long long)N);
  return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

const char* rw_last_error(void) { return g_last_error; }
int rw_version(void) { return 1; }

int rw_graph_bytes(const rw_graph_desc* desc, size_t* bytes) {
  RW_TRY(validate_desc(desc));
  RW_CHECK(bytes != nullptr, RW_EINVAL, "null bytes pointer");
  *bytes = graph_layout(*desc, nullptr, nullptr);
  return RW_OK;
}

int rw_build_graph(const rw_graph_desc* desc, const void* J_dev, int J_dtype, double beta,
                   void* graph_buf, size_t buf_bytes, hipStream_t stream, rw_graph* out) {
  RW_TRY(validate_desc(desc));
  RW_CHECK(out != nullptr && J_dev != nullptr && graph_buf != nullptr, RW_EINVAL, "null pointer argument");
  RW_CHECK(J_dtype == RW_F64 || J_dtype == RW_F32, RW_EINVAL, "J dtype must be F64 or F32");
  RW_CHECK(std::isfinite(beta) && beta >= 0.0, RW_EINVAL, "beta must be finite and >= 0 (got %g)", beta);
  size_t need = graph_layout(*desc, nullptr, nullptr);
  RW_CHECK(buf_bytes >= need, RW_EWORKSPACE, "graph buffer too small: %zu < %zu", buf_bytes, need);
  RW_CHECK((reinterpret_cast<uintptr_t>(graph_buf) & 255) == 0, RW_EINVAL, "graph buffer must be 256-byte aligned");
  rw_graph h = new rw_graph_s();
  Graph* g = &h->g;
  g->ndim = desc->ndim;
  g->nx = desc->dims[0]; g->ny = desc->dims[1]; g->nz = desc->dims[2];
  g->N = g->nx * g->ny * g->nz;
  g->conn = desc->conn;
  g->dtype = desc->dtype;
  g->weight_form = desc->weight_form;
  g->normalized = desc->normalized ? 1 : 0;
  g->beta = beta;
  static const int d2_4[2][3] = {{1, 0, 0}, {0, 1, 0}};
  static const int d2_8[4][3] = {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {1, -1, 0}};
  static const int d3_6[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const int(*dirs)[3] = g->ndim == 3 ? d3_6 : (g->conn == 8 ? d2_8 : d2_4);
  g->ndir = g->ndim == 3 ? 3 : (g->conn == 8 ? 4 : 2);
  for (int k = 0; k < g->ndir; ++k) {
    g->dx[k] = dirs[k][0]; g->dy[k] = dirs[k][1]; g->dz[k] = dirs[k][2];
    g->off[k] = dirs[k][0] + g->nx * (dirs[k][1] + g->ny * (int64_t)dirs[k][2]);
  }
  graph_layout(*desc, g, graph_buf);
  GridDev G = grid_of(g);
  k_graph_init<<<nblocks(g->N, 256), 256, 0, stream>>>(G, J_dev, J_dtype, g->J, g->scale, g->mask);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { delete h; set_error("graph init launch: %s", hipGetErrorString(e)); return RW_EHIP; }
  int st = graph_rebuild(g, stream);
  if (st != RW_OK) { delete h; return st; }
  *out = h;
  return RW_OK;
}

int rw_graph_destroy(rw_graph g) {
  delete g;
  return RW_OK;
}

int rw_graph_get_view(rw_graph h, rw_graph_view* v) {
  RW_CHECK(h != nullptr && v != nullptr, RW_EINVAL, "null argument");
  const Graph* g = &h->g;
  v->N = g->N; v->ndir = g->ndir; v->dtype = g->dtype; v->beta = g->beta;
  v->J = g->J; v->weight = g->weight; v->scale = g->scale; v->coef = g->coef; v->diag = g->diag;
  v->dinv = g->dinv; v->ghat = g->ghat; v->degree = g->degree; v->mask = g->mask; v->comp = g->comp;
  return RW_OK;
}

int rw_graph_components(rw_graph h, int64_t* n_components, hipStream_t stream) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  Graph* g = &h->g;
  RW_TRY(graph_components(g, stream));
  if (n_components) {
    RW_HIP(hipMemsetAsync(g->cc_flag + 2, 0, 2 * sizeof(int), stream));
    k_cc_count<<<nblocks(g->N, 256), 256, 0, stream>>>(g->comp, g->N, reinterpret_cast<unsigned long long*>(g->cc_flag + 2));
    RW_LAUNCH_CHECK();
    unsigned long long cnt = 0;
    RW_HIP(hipMemcpyAsync(&cnt, g->cc_flag + 2, sizeof(cnt), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipStreamSynchronize(stream));
    *n_components = (int64_t)cnt;
  }
  return RW_OK;
}

int rw_edit_graph(rw_graph h, const rw_edit* edits, int n_edits, hipStream_t stream) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr, RW_EINVAL, "null graph");
  RW_CHECK(n_edits >= 0 && (n_edits == 0 || edits != nullptr), RW_EINVAL, "bad edit list");
  Graph* g = &h->g;
  if (n_edits == 0) return RW_OK;
  // host-side validation against a copy of the presence mask, updated as the list is walked (the graph keeps
  // the host copy from its first edit on)
  if (g->hmask.size() != (size_t)g->N) {
    g->hmask.resize(g->N);
    RW_HIP(hipMemcpyAsync(g->hmask.data(), g->mask, g->N, hipMemcpyDeviceToHost, stream));
    RW_HIP(hipStreamSynchronize(stream));
  }
  std::vector<uint8_t> mask = g->hmask;
  for (int k = 0; k < n_edits; ++k) {
    const rw_edit& e = edits[k];
    switch (e.kind) {
      case RW_EDIT_SET_BETA:
        RW_CHECK(std::isfinite(e.value) && e.value >= 0.0, RW_EINVAL, "edit %d: beta must be >= 0", k);
        break;
      case RW_EDIT_SCALE_BOX:
        RW_CHECK(std::isfinite(e.value) && e.value > 0.0, RW_EINVAL, "edit %d: scale must be > 0", k);
        break;
      case RW_EDIT_SCALE_EDGES:
      case RW_EDIT_REMOVE_EDGES: {
        if (e.kind == RW_EDIT_SCALE_EDGES)
          RW_CHECK(std::isfinite(e.value) && e.value > 0.0, RW_EINVAL, "edit %d: scale must be > 0", k);
        RW_CHECK(e.n >= 0 && (e.n == 0 || e.edge_ids != nullptr), RW_EINVAL, "edit %d: bad id list", k);
        std::vector<uint8_t> seen;
        for (int64_t j = 0; j < e.n; ++j) {
          int64_t id = e.edge_ids[j];
          RW_CHECK(id >= 0 && id < g->ndir * g->N, RW_EINVAL, "edit %d: edge id %lld out of range", k, (long long)id);
          int d = (int)(id / g->N);
          int64_t t = id % g->N;
          RW_CHECK((mask[t] >> d) & 1u, RW_EINVAL, "edit %d: edge %lld is not present", k, (long long)id);
          if (e.kind == RW_EDIT_REMOVE_EDGES) mask[t] &= uint8_t(~(1u << d));
        }
        if (e.kind == RW_EDIT_SCALE_EDGES) {  // distinct ids: sort a copy
          std::vector<int64_t> ids(e.edge_ids, e.edge_ids + e.n);
          std::sort(ids.begin(), ids.end());
          for (size_t j = 1; j < ids.size(); ++j)
            RW_CHECK(ids[j] != ids[j - 1], RW_EINVAL, "edit %d: edge %lld listed twice", k, (long long)ids[j]);
        }
        break;
      }
      default:
        RW_CHECK(false, RW_EINVAL, "edit %d: unknown kind %d", k, e.kind);
    }
  }
  // apply in order
  GridDev G = grid_of(g);
  int64_t* stage = edit_stage(g);
  for (int k = 0; k < n_edits; ++k) {
    const rw_edit& e = edits[k];
    if (e.kind == RW_EDIT_SET_BETA) {
      g->beta = e.value;
    } else if (e.kind == RW_EDIT_SCALE_BOX) {
      k_scale_box<<<nblocks(g->N, 256), 256, 0, stream>>>(G, e.box_lo[0], e.box_lo[1], e.box_lo[2], e.box_hi[0],
                                                          e.box_hi[1], e.box_hi[2], e.value, g->mask, g->scale);
      RW_LAUNCH_CHECK();
    } else {
      int rem = e.kind == RW_EDIT_REMOVE_EDGES;
      for (int64_t j0 = 0; j0 < e.n; j0 += kEditStage) {
        int64_t cnt = std::min<int64_t>(kEditStage, e.n - j0);
        RW_HIP(hipMemcpyAsync(stage, e.edge_ids + j0, cnt * sizeof(int64_t), hipMemcpyHostToDevice, stream));
        k_edit_ids<<<nblocks(cnt, 256), 256, 0, stream>>>(stage, cnt, e.value, rem, g->scale);
        RW_LAUNCH_CHECK();
        // the staging area is reused by the next chunk only after this kernel has read it
        RW_HIP(hipStreamSynchronize(stream));
      }
    }
  }
  const bool mask_changed = mask != g->hmask;
  if (mask_changed) {
    g->hmask.swap(mask);
    RW_HIP(hipMemcpyAsync(g->mask, g->hmask.data(), g->N, hipMemcpyHostToDevice, stream));
  }
  RW_TRY(graph_rebuild(g, stream));
  if (mask_changed) RW_HIP(hipStreamSynchronize(stream));   // the host copy is the source of the upload
  return RW_OK;
}

}  // extern "C"
