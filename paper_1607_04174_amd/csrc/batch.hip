// Batched online solves: many images (ragged sizes, different m, C and seed sets) in one enqueue of
// device-only kernels, so that a caller can capture an interaction round into a HIP graph and replay
// it.  Per round the host validates and uploads the seeds (rw_batch_set_seeds); rw_batch_enqueue
// then launches, for all images at once: seed maps, the seed gather, the per-image reduced systems
// (Q_s^T B Q_n and Q_s^T op_ss U_hat_s), one LU per image, and a persistent reconstruction kernel
// that walks a global list of (image, node tile) work items.  Every launch reads its sizes from
// device descriptors, so replays stay valid when the seeds, S or C change between rounds (up to the
// capacities given at creation).  The reconstruction's launch shape (threads per block, nodes per
// thread) is chosen at creation by timing the candidates on the batch itself (autotuner), with the
// choice cached per batch shape for the process and, if RW_AUTOTUNE_CACHE names a file, on disk.
// Each image's basis is taken in FP64 as the exact null vector plus the other columns made orthogonal to
// it, as in the single-image solve; the constants of that correction (c_j, n_j) are computed once at
// creation, so the graphs and bases must not change while the batch is used.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <vector>

#include "rw_internal.h"

namespace rw {

constexpr int kBatchMaxC = 8;

struct BatchImg {
  GridDev G;
  int normalized;
  int m;
  int C;              // labels this round
  int C_cap;
  const double* weight;   // FP64 edge weights (ndir x N)
  const double* sums;     // [0] = 1^T D 1
  const double* cn;       // 2 m: c_j, n_j of the FP64 basis
  const double* degree;
  const void* dinv;
  const void* Q;
  const double* lambda;
  void* U;
  uint8_t* map;
  int64_t seed_off;   // first seed of this image in the round's arrays
  int64_t S;          // seeds this round (after de-duplication)
  int64_t S_cap;
  double *Qs, *GB, *Hs, *Us, *T, *R, *K, *Y, *stat;
};

struct BatchTile {
  int img;
  int pad;
  int64_t node0;
};

struct Variant {
  int threads;
  int npt;
};

struct rw_batch_impl {
  std::vector<rw_batch_image> imgs;
  int n = 0;
  int gdt = RW_F32, qdt = RW_F32;
  int64_t S_total_cap = 0;
  int64_t max_N = 0;
  int max_m = 0;
  int max_C = 1;   // largest label capacity (reconstruction tile width 4 or 8)
  // device pointers inside the caller's workspace
  BatchImg* d_desc = nullptr;
  LuJob* d_jobs = nullptr;
  int64_t* d_seed_node = nullptr;
  int32_t* d_seed_label = nullptr;
  int32_t* d_seed_img = nullptr;
  BatchTile* d_tiles = nullptr;
  int64_t* d_total = nullptr;   // seeds in the current round (device copy, read by the kernels)
  double* d_npart = nullptr;    // basis-constant partials (used at creation)
  int* d_nbad = nullptr;        // per image: a basis column in the span of the null vector
  int64_t tile_cap = 0;
  // host mirrors
  std::vector<BatchImg> desc;
  Variant var{256, 1};
  int64_t ntiles = 0;
  int64_t total_seeds = 0;
  bool tuned_now = false;
  bool have_seeds = false;
  double tune_us = 0.0;
};

static size_t batch_layout(const rw_batch_image* imgs, int n, void* base, rw_batch_impl* b) {
  Carver c(base);
  BatchImg* desc = c.take<BatchImg>(n);
  LuJob* jobs = c.take<LuJob>(n);
  int64_t S_tot = 0, tiles = 0;
  for (int i = 0; i < n; ++i) {
    S_tot += imgs[i].S_cap;
    tiles += (imgs[i].g->g.N + 63) / 64;   // enough for the smallest tile (64 nodes)
  }
  int64_t* sn = c.take<int64_t>(std::max<int64_t>(S_tot, 1));
  int32_t* sl = c.take<int32_t>(std::max<int64_t>(S_tot, 1));
  int32_t* si = c.take<int32_t>(std::max<int64_t>(S_tot, 1));
  BatchTile* tl = c.take<BatchTile>(std::max<int64_t>(tiles, 1));
  int64_t* tot = c.take<int64_t>(1);
  size_t npc = 1;
  for (int i = 0; i < n; ++i) npc = std::max(npc, null_stats_partial_count(imgs[i].g->g.N, imgs[i].m));
  double* npart = c.take<double>(npc);
  int* nbad = c.take<int>((size_t)n);
  if (b) {
    b->d_npart = npart;
    b->d_nbad = nbad;
    b->d_desc = desc; b->d_jobs = jobs; b->d_seed_node = sn; b->d_seed_label = sl; b->d_seed_img = si;
    b->d_tiles = tl; b->d_total = tot; b->tile_cap = tiles; b->S_total_cap = S_tot;
    b->desc.resize(n);
  }
  for (int i = 0; i < n; ++i) {
    const rw_batch_image& im = imgs[i];
    const int64_t N = im.g->g.N, S = im.S_cap, m = im.m, Cc = im.C_cap;
    uint8_t* map = c.take<uint8_t>(N);
    double* Qs = c.take<double>(S * m);
    double* GB = c.take<double>(S * m);
    double* Hs = c.take<double>(S * Cc);
    double* Us = c.take<double>(S * Cc);
    double* T = c.take<double>(m * m);
    double* R = c.take<double>(m * Cc);
    double* K = c.take<double>(m * m);
    double* Y = c.take<double>(m * Cc);
    double* st = c.take<double>(8);
    double* cn = c.take<double>(2 * m);
    if (b) {
      BatchImg& d = b->desc[i];
      const Graph* g = &im.g->g;
      d.G = grid_of(g);
      d.normalized = g->normalized;
      d.m = im.m;
      d.C = 0;
      d.C_cap = im.C_cap;
      d.weight = g->weight; d.sums = g->sums; d.cn = cn; d.degree = g->degree; d.dinv = g->dinv;
      d.Q = im.Q; d.lambda = im.lambda; d.U = im.U; d.map = map;
      d.seed_off = 0; d.S = 0; d.S_cap = S;
      d.Qs = Qs; d.GB = GB; d.Hs = Hs; d.Us = Us; d.T = T; d.R = R; d.K = K; d.Y = Y; d.stat = st;
    }
  }
  return c.used;
}

// ---------------------------------------------------------------------------------------------
// kernels (all images at once; sizes from the device descriptors)
// ---------------------------------------------------------------------------------------------
__global__ void k_b_clear_maps(const BatchImg* D, int n) {
  const BatchImg& d = D[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.G.N; i += (int64_t)gridDim.x * blockDim.x)
    d.map[i] = 0;
}

__global__ void k_b_set_maps(const BatchImg* D, const int64_t* node, const int32_t* label, const int32_t* img,
                             const int64_t* total) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= *total) return;
  D[img[k]].map[node[k]] = (uint8_t)(label[k] + 1);
}

template <typename TQ>
__global__ void k_b_gather(const BatchImg* D, const int64_t* node, const int32_t* label, const int32_t* img,
                           const int64_t* total) {
  const int64_t gk = blockIdx.x;
  if (gk >= *total) return;
  const BatchImg& d = D[img[gk]];
  gather_seed_row<TQ>(d.G, d.normalized, d.weight, d.degree, d.sums, static_cast<const TQ*>(d.Q), nullptr, d.m, d.map,
                      node[gk], d.C, d.cn, gk - d.seed_off, d.S_cap, d.Qs, d.GB, d.Hs, d.Us, nullptr, nullptr);
}

// T = Q_s^T GB and R = Q_s^T Hs per image (FP64, summed over the image's S seeds in order), then
// K = diag(lambda) - T and the right-hand side Y = R.  32 x 32 tiles of the output per workgroup (the single
// solve's code): workgroup x runs over the tiles of image y.
__global__ __launch_bounds__(256) void k_b_reduced(const BatchImg* D, LuJob* jobs) {
  __shared__ double sA[kRedTile * 33], sB[kRedTile * 33];
  const BatchImg& d = D[blockIdx.y];
  const int m = d.m, C = d.C;
  const int64_t S = d.S, ld = d.S_cap;
  const int tr = (m + kRedTile - 1) / kRedTile, tc = (m + C + kRedTile - 1) / kRedTile;
  for (int t = blockIdx.x; t < tr * tc; t += gridDim.x)
    reduced_tile(t % tr, t / tr, m, C, S, ld, d.Qs, d.GB, d.Hs, d.lambda, 0.0, d.K, d.Y, sA, sB);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    LuJob jb;
    jb.A = d.K; jb.B = d.Y; jb.stat = d.stat; jb.n = m; jb.nrhs = C;
    jobs[blockIdx.y] = jb;
  }
}

// after the batched LU: the coefficients of the stored columns and the null vector's term per image
__global__ __launch_bounds__(256) void k_b_coeffs(const BatchImg* D) {
  const BatchImg& d = D[blockIdx.x];
  solve_coeffs_block(d.Y, d.m, d.C, d.cn, ghat_scaled64(d.sums, d.normalized, d.G.N));
}

// persistent reconstruction over the (image, tile) list: U = D^{-1/2} sum_{j>=1} Q_j Y_j + kappa on non-seeds,
// one-hot on seeds.  Y's rows 1..m-1 (x CB, zero-padded labels) and kappa (row 0) are staged in LDS per tile;
// each thread owns NPT nodes and keeps 4 * NPT loads of Q in flight (the j loop is unrolled by 4), so the
// pass over Q is bandwidth-bound.
template <typename TQ, typename TU, int NPT, int CB>
__global__ __launch_bounds__(512) void k_b_reconstruct(const BatchImg* D, const BatchTile* tiles, int64_t ntiles) {
  using CT = typename Elem<TQ>::C;
  extern __shared__ char smem[];
  CT* sY = reinterpret_cast<CT*>(smem);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    const BatchImg& d = D[tl.img];
    const int m = d.m - 1, C = d.C;   // columns 1 .. d.m - 1
    CT* sK = sY + m * CB;
    __syncthreads();
    for (int q = threadIdx.x; q < d.m * CB; q += blockDim.x) {
      const int j = q / CB, c = q % CB;
      const CT v = c < C ? (CT)d.Y[j + (int64_t)c * d.m] : CT(0);
      if (j == 0) sK[c] = v;
      else sY[(j - 1) * CB + c] = v;
    }
    __syncthreads();
    const int64_t N = d.G.N;
    const TQ* Q = static_cast<const TQ*>(d.Q) + N;
    int64_t ii[NPT];
    bool ok[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int64_t i = tl.node0 + threadIdx.x + (int64_t)r * blockDim.x;
      ok[r] = i < N;
      ii[r] = ok[r] ? i : tl.node0;      // a valid node for the (discarded) loads of an idle slot
    }
    CT acc[NPT][CB];
#pragma unroll
    for (int r = 0; r < NPT; ++r)
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[r][c] = CT(0);
    int j = 0;
    for (; j + 4 <= m; j += 4) {
      CT q[4][NPT];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < NPT; ++r) q[u][r] = Elem<TQ>::ld(Q, (int64_t)(j + u) * N + ii[r]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          const CT y = sY[(j + u) * CB + c];
#pragma unroll
          for (int r = 0; r < NPT; ++r) acc[r][c] = fma(q[u][r], y, acc[r][c]);
        }
    }
    for (; j < m; ++j) {
#pragma unroll
      for (int r = 0; r < NPT; ++r) {
        const CT q = Elem<TQ>::ld(Q, (int64_t)j * N + ii[r]);
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[r][c] = fma(q, sY[j * CB + c], acc[r][c]);
      }
    }
    TU* U = static_cast<TU*>(d.U);
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      if (!ok[r]) continue;
      const int64_t i = ii[r];
      const int ml = d.map[i];
      const CT sc = d.normalized ? (CT) static_cast<const TU*>(d.dinv)[i] : CT(1);
      const bool live = !d.normalized || sc > CT(0);
#pragma unroll
      for (int c = 0; c < CB; ++c)
        if (c < C)
          U[(int64_t)c * N + i] = ml ? (ml - 1 == c ? TU(1) : TU(0)) : (TU)(sc * acc[r][c] + (live ? sK[c] : CT(0)));
    }
  }
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
static const Variant kVariants[] = {{128, 1}, {256, 1}, {256, 2}, {256, 4}, {512, 1}, {512, 2}};

static std::mutex g_tune_mu;
static std::map<std::string, Variant> g_tune_cache;
static bool g_tune_loaded = false;

static void load_tune_cache() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("RW_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string key;
  int th = 0, npt = 0;
  while (f >> key >> th >> npt) g_tune_cache[key] = Variant{th, npt};
}

static void save_tune_cache() {
  const char* path = std::getenv("RW_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream f(path);
  for (auto& kv : g_tune_cache) f << kv.first << " " << kv.second.threads << " " << kv.second.npt << "\n";
}

static int build_tiles(rw_batch_impl* b, Variant v, hipStream_t s) {
  std::vector<BatchTile> tl;
  const int64_t span = (int64_t)v.threads * v.npt;
  for (int i = 0; i < b->n; ++i) {
    const int64_t N = b->imgs[i].g->g.N;
    for (int64_t n0 = 0; n0 < N; n0 += span) tl.push_back(BatchTile{i, 0, n0});
  }
  RW_CHECK((int64_t)tl.size() <= b->tile_cap, RW_EINVAL, "tile list exceeds its capacity");
  RW_HIP(hipMemcpyAsync(b->d_tiles, tl.data(), tl.size() * sizeof(BatchTile), hipMemcpyHostToDevice, s));
  RW_HIP(hipStreamSynchronize(s));
  b->ntiles = (int64_t)tl.size();
  return RW_OK;
}

template <typename TQ, typename TU, int CB>
static int launch_recon_cb(const rw_batch_impl* b, Variant v, hipStream_t s) {
  const size_t sh = (size_t)b->max_m * CB * sizeof(typename Elem<TQ>::C);   // (m - 1) rows + kappa
  const unsigned grid = (unsigned)std::min<int64_t>(b->ntiles, 2048);
  if (grid == 0) return RW_OK;
  if (v.npt == 1) k_b_reconstruct<TQ, TU, 1, CB><<<grid, v.threads, sh, s>>>(b->d_desc, b->d_tiles, b->ntiles);
  else if (v.npt == 2) k_b_reconstruct<TQ, TU, 2, CB><<<grid, v.threads, sh, s>>>(b->d_desc, b->d_tiles, b->ntiles);
  else k_b_reconstruct<TQ, TU, 4, CB><<<grid, v.threads, sh, s>>>(b->d_desc, b->d_tiles, b->ntiles);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

template <typename TQ, typename TU>
static int launch_recon_t(const rw_batch_impl* b, Variant v, hipStream_t s) {
  return b->max_C <= 4 ? launch_recon_cb<TQ, TU, 4>(b, v, s) : launch_recon_cb<TQ, TU, 8>(b, v, s);
}

static int launch_recon(const rw_batch_impl* b, Variant v, hipStream_t s) {
  if (b->gdt == RW_F64) {
    if (b->qdt == RW_F64) return launch_recon_t<double, double>(b, v, s);
    if (b->qdt == RW_F32) return launch_recon_t<float, double>(b, v, s);
    return launch_recon_t<uint16_t, double>(b, v, s);
  }
  if (b->qdt == RW_F64) return launch_recon_t<double, float>(b, v, s);
  if (b->qdt == RW_F32) return launch_recon_t<float, float>(b, v, s);
  return launch_recon_t<uint16_t, float>(b, v, s);
}

static int autotune(rw_batch_impl* b, hipStream_t s) {
  std::ostringstream key;
  int64_t work = 0;
  for (auto& im : b->imgs) work += im.g->g.N * (int64_t)im.m;
  key << "batch_n" << b->n << "_Nm" << work << "_g" << b->gdt << "_q" << b->qdt << "_c" << b->max_C;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache();
    auto it = g_tune_cache.find(key.str());
    if (it != g_tune_cache.end()) {
      b->var = it->second;
      return build_tiles(b, b->var, s);
    }
  }
  // the descriptors hold C = 0 until the first seeds arrive, so the timed launches write nothing;
  // their cost is the read of every image's basis, which is what the launch shape changes
  hipEvent_t e0, e1;
  RW_HIP(hipEventCreate(&e0));
  RW_HIP(hipEventCreate(&e1));
  double best = INFINITY;
  Variant bestv = kVariants[0];
  auto t0 = std::chrono::steady_clock::now();
  for (const Variant& v : kVariants) {
    RW_TRY(build_tiles(b, v, s));
    RW_TRY(launch_recon(b, v, s));   // warm-up
    RW_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) RW_TRY(launch_recon(b, v, s));
    RW_HIP(hipEventRecord(e1, s));
    RW_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    RW_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) { best = ms; bestv = v; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->tune_us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  b->tuned_now = true;
  b->var = bestv;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key.str()] = bestv;
    save_tune_cache();
  }
  return build_tiles(b, b->var, s);
}

}  // namespace rw

using namespace rw;

struct rw_batch_s {
  rw_batch_impl b;
};

extern "C" {

int rw_batch_workspace_bytes(const rw_batch_image* imgs, int n, size_t* bytes) {
  RW_CHECK(imgs != nullptr && n >= 1 && n <= 65535 && bytes != nullptr, RW_EINVAL, "bad argument");
  for (int i = 0; i < n; ++i)
    RW_CHECK(imgs[i].g != nullptr && imgs[i].m >= 2 && imgs[i].m <= 1024 && imgs[i].S_cap >= 1 && imgs[i].C_cap >= 1 &&
                 imgs[i].C_cap <= kBatchMaxC, RW_EINVAL, "image %d: bad sizes", i);
  *bytes = batch_layout(imgs, n, nullptr, nullptr);
  return RW_OK;
}

int rw_batch_create(const rw_batch_image* imgs, int n, void* work, size_t work_bytes, hipStream_t stream,
                    rw_batch* out) {
  RW_NOT_CAPTURING(stream);
  size_t need = 0;
  RW_TRY(rw_batch_workspace_bytes(imgs, n, &need));
  RW_CHECK(work != nullptr && out != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "batch workspace too small: %zu < %zu", work_bytes, need);
  const int gdt = imgs[0].g->g.dtype, qdt = imgs[0].q_dtype;
  RW_CHECK(qdt == RW_F64 || qdt == RW_F32 || qdt == RW_BF16, RW_EINVAL,
           "the batched solve takes RW_F64, RW_F32 or RW_BF16 bases (pass a pair form's plain block with RW_BF16)");
  for (int i = 0; i < n; ++i) {
    const rw_batch_image& im = imgs[i];
    RW_CHECK(im.g->g.dtype == gdt && im.q_dtype == qdt, RW_EINVAL, "all images need the same graph and Q types");
    RW_CHECK(im.Q != nullptr && im.lambda != nullptr && im.U != nullptr, RW_EINVAL, "image %d: null pointer", i);
    RW_CHECK(im.m <= im.g->g.N, RW_EINVAL, "image %d: m > N", i);
    RW_CHECK((size_t)im.m * kBatchMaxC * 8 <= 65536, RW_EINVAL, "image %d: m too large", i);
  }
  rw_batch h = new rw_batch_s();
  rw_batch_impl* b = &h->b;
  b->imgs.assign(imgs, imgs + n);
  b->n = n;
  b->gdt = gdt;
  b->qdt = qdt;
  for (int i = 0; i < n; ++i) {
    b->max_N = std::max<int64_t>(b->max_N, imgs[i].g->g.N);
    b->max_m = std::max(b->max_m, imgs[i].m);
    b->max_C = std::max(b->max_C, imgs[i].C_cap);
  }
  batch_layout(imgs, n, work, b);
  hipError_t e = hipMemcpyAsync(b->d_desc, b->desc.data(), n * sizeof(BatchImg), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    delete h;
    set_error("batch descriptors: %s", hipGetErrorString(e));
    return RW_EHIP;
  }
  // basis constants of every image (one pass over each basis), checked before the batch is handed out
  int st = RW_OK;
  std::vector<int> nbad((size_t)n, 0);
  if (hipMemsetAsync(b->d_nbad, 0, n * sizeof(int), stream) != hipSuccess) st = RW_EHIP;
  for (int i = 0; i < n && st == RW_OK; ++i)
    st = null_stats(&imgs[i].g->g, imgs[i].Q, qdt, imgs[i].m, b->d_npart, const_cast<double*>(b->desc[i].cn),
                    b->d_nbad + i, stream);
  if (st == RW_OK && (hipMemcpyAsync(nbad.data(), b->d_nbad, n * sizeof(int), hipMemcpyDeviceToHost, stream) !=
                          hipSuccess ||
                      hipStreamSynchronize(stream) != hipSuccess)) {
    set_error("batch basis constants: %s", hipGetErrorString(hipGetLastError()));
    st = RW_EHIP;
  }
  for (int i = 0; i < n && st == RW_OK; ++i)
    if (nbad[i]) {
      set_error("image %d: basis column %d lies in the span of the null vector (column 0)", i, nbad[i]);
      st = RW_EINVAL;
    }
  if (st == RW_OK) st = autotune(b, stream);
  if (st != RW_OK) {
    delete h;
    return st;
  }
  *out = h;
  return RW_OK;
}

int rw_batch_destroy(rw_batch h) {
  delete h;
  return RW_OK;
}

int rw_batch_info(rw_batch h, int* threads, int* nodes_per_thread, int* tuned_now, double* tune_us) {
  RW_CHECK(h != nullptr, RW_EINVAL, "null batch");
  if (threads) *threads = h->b.var.threads;
  if (nodes_per_thread) *nodes_per_thread = h->b.var.npt;
  if (tuned_now) *tuned_now = h->b.tuned_now ? 1 : 0;
  if (tune_us) *tune_us = h->b.tune_us;
  return RW_OK;
}

int rw_batch_set_seeds(rw_batch h, const int* C, const int64_t* seed_off, const int64_t* seed_node,
                       const int32_t* seed_label, hipStream_t stream) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr && C != nullptr && seed_off != nullptr && seed_node != nullptr && seed_label != nullptr,
           RW_EINVAL, "null argument");
  rw_batch_impl* b = &h->b;
  std::vector<BatchImg> nd = b->desc;   // committed only when every image validates
  std::vector<int64_t> nodes;
  std::vector<int32_t> labels, imgid;
  nodes.reserve(b->S_total_cap);
  for (int i = 0; i < b->n; ++i) {
    BatchImg& d = nd[i];
    const int64_t N = d.G.N;
    RW_CHECK(C[i] >= 1 && C[i] <= d.C_cap, RW_EINVAL, "image %d: C = %d exceeds its capacity %d", i, C[i], d.C_cap);
    RW_CHECK(seed_off[i + 1] > seed_off[i], RW_EINVAL, "image %d: at least one seed is required", i);
    std::vector<std::pair<int64_t, int32_t>> v;
    for (int64_t k = seed_off[i]; k < seed_off[i + 1]; ++k) {
      RW_CHECK(seed_node[k] >= 0 && seed_node[k] < N, RW_EINVAL, "image %d: seed node out of range", i);
      RW_CHECK(seed_label[k] >= 0 && seed_label[k] < C[i], RW_EINVAL, "image %d: seed label out of range", i);
      v.push_back({seed_node[k], seed_label[k]});
    }
    std::sort(v.begin(), v.end());
    d.seed_off = (int64_t)nodes.size();
    for (size_t k = 0; k < v.size(); ++k) {
      if (k && v[k].first == v[k - 1].first) {
        RW_CHECK(v[k].second == v[k - 1].second, RW_EINVAL, "image %d: node %lld seeded with two labels", i,
                 (long long)v[k].first);
        continue;
      }
      nodes.push_back(v[k].first);
      labels.push_back(v[k].second);
      imgid.push_back(i);
    }
    d.S = (int64_t)nodes.size() - d.seed_off;
    RW_CHECK(d.S <= d.S_cap, RW_EINVAL, "image %d: %lld seeds exceed the capacity %lld", i, (long long)d.S,
             (long long)d.S_cap);
    RW_CHECK(d.S < N, RW_EINVAL, "image %d: every node is a seed", i);
    d.C = C[i];
  }
  b->desc.swap(nd);
  b->total_seeds = (int64_t)nodes.size();
  b->have_seeds = true;
  RW_HIP(hipMemcpyAsync(b->d_seed_node, nodes.data(), nodes.size() * sizeof(int64_t), hipMemcpyHostToDevice, stream));
  RW_HIP(hipMemcpyAsync(b->d_seed_label, labels.data(), labels.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  RW_HIP(hipMemcpyAsync(b->d_seed_img, imgid.data(), imgid.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  RW_HIP(hipMemcpyAsync(b->d_desc, b->desc.data(), b->n * sizeof(BatchImg), hipMemcpyHostToDevice, stream));
  RW_HIP(hipMemcpyAsync(b->d_total, &b->total_seeds, sizeof(int64_t), hipMemcpyHostToDevice, stream));
  RW_HIP(hipStreamSynchronize(stream));
  return RW_OK;
}

int rw_batch_enqueue(rw_batch h, hipStream_t stream) {
  RW_CHECK(h != nullptr, RW_EINVAL, "null batch");
  rw_batch_impl* b = &h->b;
  RW_CHECK(b->have_seeds, RW_EINVAL, "rw_batch_set_seeds must come before the first enqueue");
  // Every launch shape below depends on the capacities only; this round's sizes are read on the
  // device, so a captured graph of this call stays valid for every later round.
  const int64_t cap = std::max<int64_t>(b->S_total_cap, 1);
  k_b_clear_maps<<<dim3((unsigned)std::min<int64_t>(nblocks(b->max_N, 256), 1024), b->n), 256, 0, stream>>>(b->d_desc,
                                                                                                             b->n);
  RW_LAUNCH_CHECK();
  k_b_set_maps<<<nblocks(cap, 256), 256, 0, stream>>>(b->d_desc, b->d_seed_node, b->d_seed_label, b->d_seed_img,
                                                      b->d_total);
  RW_LAUNCH_CHECK();
#define RW_BGATHER(TQ)                                                                                  \
  k_b_gather<TQ><<<(unsigned)cap, 256, 0, stream>>>(b->d_desc, b->d_seed_node, b->d_seed_label, b->d_seed_img, \
                                                    b->d_total)
  if (b->qdt == RW_F64) RW_BGATHER(double);
  else if (b->qdt == RW_F32) RW_BGATHER(float);
  else RW_BGATHER(uint16_t);
#undef RW_BGATHER
  RW_LAUNCH_CHECK();
  const int64_t per_img = (int64_t)((b->max_m + kRedTile - 1) / kRedTile) *
                          ((b->max_m + kBatchMaxC + kRedTile - 1) / kRedTile);   // tiles of the largest image
  k_b_reduced<<<dim3((unsigned)per_img, b->n), 256, 0, stream>>>(b->d_desc, b->d_jobs);
  RW_LAUNCH_CHECK();
  RW_TRY(lu_solve_batched(b->d_jobs, b->n, stream));
  k_b_coeffs<<<b->n, 256, 0, stream>>>(b->d_desc);
  RW_LAUNCH_CHECK();
  RW_TRY(launch_recon(b, b->var, stream));
  return RW_OK;
}

int rw_batch_status(rw_batch h, double* min_pivot, hipStream_t stream) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr && min_pivot != nullptr, RW_EINVAL, "null argument");
  rw_batch_impl* b = &h->b;
  double worst = INFINITY;
  for (int i = 0; i < b->n; ++i) {
    double st = 0.0;
    RW_HIP(hipMemcpyAsync(&st, b->desc[i].stat, sizeof(double), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipStreamSynchronize(stream));
    worst = std::min(worst, st);
  }
  *min_pivot = worst;
  RW_CHECK(worst > 0.0, RW_ESINGULAR, "a reduced seed system of the batch is singular");
  return RW_OK;
}

}  // extern "C"
