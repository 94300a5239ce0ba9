// Vertex aggregation (Sec. III-C) over regular blocks of s x s (x s) voxels, the last ones clipped at the
// border: the aggregated graph (the block grid, same connectivity, the weight between two blocks the sum of
// the weights of the edges joining them, so that its Laplacian is P^T L P for the 0/1 assignment P), the
// transfer of the stored eigenvectors by eq. (33),
//   Delta(x) = sum over the edge neighbours x' of sum_y |eta(x, y) - eta(x', y)|  (2 per neighbour in another
//              block: eta(x, y) = 1 for x's block),
//   q_bar_y  = sum_{x in y} Delta(x) q_x / |y|                                   (eta_bar(x, y) = 1 / |y|),
// after which rw_update_eig's diagonal update on the aggregated graph orthonormalizes the columns in order
// against its null vector and gives their normalized-cut values, and the propagation U_x = U_bar_{y(x)}.
#include <algorithm>
#include <map>

#include "rw_internal.h"

namespace rw {

struct AggDims {
  int64_t nx, ny, nz, N;        // fine grid
  int64_t cx, cy, cz, Nc;       // block grid
  int s;
};

static AggDims agg_dims(const Graph* g, int s) {
  AggDims a;
  a.nx = g->nx; a.ny = g->ny; a.nz = g->nz; a.N = g->N; a.s = s;
  a.cx = (g->nx + s - 1) / s;
  a.cy = (g->ny + s - 1) / s;
  a.cz = g->ndim == 3 ? (g->nz + s - 1) / s : 1;
  a.Nc = a.cx * a.cy * a.cz;
  return a;
}

__device__ __forceinline__ int64_t block_of(const AggDims& a, int64_t x, int64_t y, int64_t z) {
  return x / a.s + a.cx * (y / a.s + a.cy * (z / a.s));
}

// one thread per (block yc, coarse forward direction d): the summed weights of the fine edges, in either
// direction, from a vertex of yc to a vertex of the block yc + offset(d), the vertices of yc in order
__global__ void k_agg_weights(GridDev G, AggDims a, const double* weight, double* cscale) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= a.Nc * G.ndir) return;
  const int d = (int)(t / a.Nc);
  const int64_t yc = t % a.Nc;
  const int64_t bx = yc % a.cx, by = (yc / a.cx) % a.cy, bz = yc / (a.cx * a.cy);
  const int64_t tx = bx + G.dx[d], ty = by + G.dy[d], tz = bz + G.dz[d];
  double sum = 0.0;
  if (tx >= 0 && tx < a.cx && ty >= 0 && ty < a.cy && tz >= 0 && tz < a.cz) {
    const int64_t target = tx + a.cx * (ty + a.cy * tz);
    const int64_t z0 = bz * a.s, z1 = a.nz > 1 ? std::min(a.nz, z0 + a.s) : 1;
    const int64_t y0 = by * a.s, y1 = std::min(a.ny, y0 + a.s);
    const int64_t x0 = bx * a.s, x1 = std::min(a.nx, x0 + a.s);
    for (int64_t z = z0; z < z1; ++z)
      for (int64_t y = y0; y < y1; ++y)
        for (int64_t x = x0; x < x1; ++x) {
          const int64_t i = x + G.nx * (y + G.ny * z);
          for (int e = 0; e < G.ndir; ++e) {
            // forward edge of i (head i + off) and backward edge (tail i - off)
            for (int sgn = 1; sgn >= -1; sgn -= 2) {
              const int64_t hx = x + sgn * G.dx[e], hy = y + sgn * G.dy[e], hz = z + sgn * G.dz[e];
              if (hx < 0 || hx >= G.nx || hy < 0 || hy >= G.ny || hz < 0 || hz >= G.nz) continue;
              if (block_of(a, hx, hy, hz) != target) continue;
              const int64_t tail = sgn > 0 ? i : i - G.off[e];
              sum += weight[(int64_t)e * G.N + tail];
            }
          }
        }
  }
  cscale[t] = sum;
}

// Delta(x) = 2 x the number of present edges of x whose other end lies in another block
__global__ void k_agg_delta(GridDev G, AggDims a, const uint8_t* mask, double* delta) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  const int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / (G.nx * G.ny);
  const int64_t b = block_of(a, x, y, z);
  double c = 0.0;
  for (int e = 0; e < G.ndir; ++e) {
    if (head_in(G, x, y, z, e) && ((mask[i] >> e) & 1u) &&
        block_of(a, x + G.dx[e], y + G.dy[e], z + G.dz[e]) != b)
      c += 2.0;
    if (tail_in(G, x, y, z, e)) {
      const int64_t t = i - G.off[e];
      if (((mask[t] >> e) & 1u) && block_of(a, x - G.dx[e], y - G.dy[e], z - G.dz[e]) != b) c += 2.0;
    }
  }
  delta[i] = c;
}

// one thread per (block y, column j): q_bar(y, j) = sum_{x in y} Delta(x) q(x, j) / |y|, in FP64, in order
template <typename TQ>
__global__ void k_agg_basis(AggDims a, const double* delta, const TQ* Q, int m, TQ* Qc) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= a.Nc * m) return;
  const int64_t yc = t % a.Nc;
  const int j = (int)(t / a.Nc);
  const int64_t bx = yc % a.cx, by = (yc / a.cx) % a.cy, bz = yc / (a.cx * a.cy);
  const int64_t z0 = bz * a.s, z1 = a.nz > 1 ? std::min(a.nz, z0 + a.s) : 1;
  const int64_t y0 = by * a.s, y1 = std::min(a.ny, y0 + a.s);
  const int64_t x0 = bx * a.s, x1 = std::min(a.nx, x0 + a.s);
  const TQ* q = Q + (int64_t)j * a.N;
  double sum = 0.0;
  for (int64_t z = z0; z < z1; ++z)
    for (int64_t y = y0; y < y1; ++y)
      for (int64_t x = x0; x < x1; ++x) {
        const int64_t i = x + a.nx * (y + a.ny * z);
        sum += delta[i] * (double)Elem<TQ>::ld(q, i);
      }
  const double size = (double)((z1 - z0) * (y1 - y0) * (x1 - x0));
  Elem<TQ>::st(Qc + (int64_t)j * a.Nc, yc, (typename Elem<TQ>::C)(sum / size));
}

template <typename TU>
__global__ void k_prolong(AggDims a, const TU* Uc, int C, TU* U) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= a.N || c >= C) return;
  const int64_t x = i % a.nx, y = (i / a.nx) % a.ny, z = i / (a.nx * a.ny);
  U[(int64_t)c * a.N + i] = Uc[(int64_t)c * a.Nc + block_of(a, x, y, z)];
}

}  // namespace rw

using namespace rw;

extern "C" {

int rw_aggregate_desc(rw_graph h, int s, rw_graph_desc* desc) {
  RW_CHECK(h != nullptr && desc != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(s >= 1, RW_EINVAL, "block size %d must be >= 1", s);
  const Graph* g = &h->g;
  const AggDims a = agg_dims(g, s);
  RW_CHECK(a.Nc >= 2, RW_EINVAL, "blocks of %d leave fewer than two super-vertices", s);
  desc->ndim = g->ndim;
  desc->dims[0] = a.cx;
  desc->dims[1] = a.cy;
  desc->dims[2] = a.cz;
  desc->conn = g->conn;
  desc->dtype = g->dtype;
  desc->weight_form = g->weight_form;
  desc->normalized = g->normalized;
  return RW_OK;
}

int rw_aggregate_workspace_bytes(rw_graph h, int s, size_t* bytes) {
  RW_CHECK(h != nullptr && bytes != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(s >= 1, RW_EINVAL, "block size %d must be >= 1", s);
  const Graph* g = &h->g;
  const AggDims a = agg_dims(g, s);
  *bytes = ((size_t)a.Nc * (1 + g->ndir) + (size_t)g->N) * sizeof(double) + 512;
  return RW_OK;
}

int rw_aggregate_graph(rw_graph h, int s, void* coarse_buf, size_t coarse_bytes, void* work, size_t work_bytes,
                       hipStream_t stream, rw_graph* coarse) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr && coarse_buf != nullptr && work != nullptr && coarse != nullptr, RW_EINVAL,
           "null argument");
  rw_graph_desc d;
  RW_TRY(rw_aggregate_desc(h, s, &d));
  size_t need = 0;
  RW_TRY(rw_aggregate_workspace_bytes(h, s, &need));
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "aggregation workspace too small: %zu < %zu", work_bytes, need);
  const Graph* g = &h->g;
  const AggDims a = agg_dims(g, s);
  double* zeros = static_cast<double*>(work);
  double* cscale = zeros + ((a.Nc + 31) / 32) * 32;
  RW_TRY(fill_i32(reinterpret_cast<int*>(zeros), 2 * a.Nc, 0, stream));
  k_agg_weights<<<nblocks(a.Nc * g->ndir, 256), 256, 0, stream>>>(grid_of(g), a, g->weight, cscale);
  RW_LAUNCH_CHECK();
  // intensities 0 (every base weight exp(0) = 1), then the summed weights as per-edge scales
  RW_TRY(rw_build_graph(&d, zeros, RW_F64, g->beta, coarse_buf, coarse_bytes, stream, coarse));
  const int st = rw_graph_set_scale(*coarse, cscale, stream);
  if (st != RW_OK) {
    rw_graph_destroy(*coarse);
    *coarse = nullptr;
    return st;
  }
  return RW_OK;
}

int rw_aggregate_basis(rw_graph h, int s, const void* Q, int q_dtype, int m, void* Qc, void* work, size_t work_bytes,
                       hipStream_t stream) {
  RW_CHECK(h != nullptr && Q != nullptr && Qc != nullptr && work != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(q_dtype == RW_F64 || q_dtype == RW_F32, RW_EINVAL, "the transfer takes F64 or F32 bases");
  RW_CHECK(m >= 1, RW_EINVAL, "m must be >= 1");
  size_t need = 0;
  RW_TRY(rw_aggregate_workspace_bytes(h, s, &need));
  RW_CHECK(work_bytes >= need, RW_EWORKSPACE, "aggregation workspace too small: %zu < %zu", work_bytes, need);
  const Graph* g = &h->g;
  const AggDims a = agg_dims(g, s);
  RW_CHECK(a.Nc >= 2, RW_EINVAL, "blocks of %d leave fewer than two super-vertices", s);
  double* delta = static_cast<double*>(work);
  k_agg_delta<<<nblocks(g->N, 256), 256, 0, stream>>>(grid_of(g), a, g->mask, delta);
  RW_LAUNCH_CHECK();
  if (q_dtype == RW_F64)
    k_agg_basis<double><<<nblocks(a.Nc * m, 256), 256, 0, stream>>>(a, delta, (const double*)Q, m, (double*)Qc);
  else
    k_agg_basis<float><<<nblocks(a.Nc * m, 256), 256, 0, stream>>>(a, delta, (const float*)Q, m, (float*)Qc);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

int rw_aggregate_seeds(rw_graph h, int s, const int64_t* seed_node, const int32_t* seed_label, int64_t S,
                       int64_t* out_node, int32_t* out_label, int64_t* S_out) {
  RW_CHECK(h != nullptr && seed_node != nullptr && seed_label != nullptr && out_node != nullptr &&
               out_label != nullptr && S_out != nullptr,
           RW_EINVAL, "null argument");
  RW_CHECK(s >= 1 && S >= 0, RW_EINVAL, "bad sizes");
  const Graph* g = &h->g;
  const AggDims a = agg_dims(g, s);
  std::map<int64_t, int32_t> lab;
  for (int64_t k = 0; k < S; ++k) {
    const int64_t v = seed_node[k];
    RW_CHECK(v >= 0 && v < g->N, RW_EINVAL, "seed %lld: node %lld out of range", (long long)k, (long long)v);
    const int64_t x = v % g->nx, y = (v / g->nx) % g->ny, z = v / (g->nx * g->ny);
    const int64_t b = x / s + a.cx * (y / s + a.cy * (z / s));
    auto it = lab.find(b);
    if (it == lab.end()) lab.emplace(b, seed_label[k]);
    else RW_CHECK(it->second == seed_label[k], RW_EINVAL, "block %lld holds seeds of labels %d and %d",
                  (long long)b, it->second, seed_label[k]);
  }
  int64_t n = 0;
  for (const auto& kv : lab) {
    out_node[n] = kv.first;
    out_label[n] = kv.second;
    ++n;
  }
  *S_out = n;
  return RW_OK;
}

int rw_prolong(rw_graph h, int s, const void* Uc, int C, void* U, hipStream_t stream) {
  RW_CHECK(h != nullptr && Uc != nullptr && U != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(s >= 1 && C >= 1 && C <= 65535, RW_EINVAL, "bad sizes");
  const Graph* g = &h->g;
  const AggDims a = agg_dims(g, s);
  const dim3 grid(nblocks(g->N, 256), (unsigned)C);
  if (g->dtype == RW_F64) k_prolong<double><<<grid, 256, 0, stream>>>(a, (const double*)Uc, C, (double*)U);
  else k_prolong<float><<<grid, 256, 0, stream>>>(a, (const float*)Uc, C, (float*)U);
  RW_LAUNCH_CHECK();
  return RW_OK;
}

}  // extern "C"
