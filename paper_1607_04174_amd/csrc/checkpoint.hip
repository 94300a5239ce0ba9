// Checkpoint of the offline phase (Sec. II-B: the eigenpairs are computed once, offline, and every online
// solve and update starts from them).  A file holds a fixed header and the raw eigenpairs:
//   rw_eig_header (128 bytes, little-endian) | Q (N x m column-major, q_dtype; N x (8 + m) BF16 for the
//   pair form) | lambda (m FP64)
// The header records the grid, the operator's form and a 64-bit FNV-1a hash of the FP64 edge weights
// (ndir x N, 0 where an edge is absent), so a basis is loaded only into a graph whose operator it was
// computed for.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rw_internal.h"

namespace rw {

static const char kMagic[8] = {'R', 'W', 'E', 'I', 'G', 'v', '1', '\0'};
static_assert(sizeof(rw_eig_header) == 128, "checkpoint header layout");

// FNV-1a over the graph's FP64 weight plane (read back in chunks)
static int weight_hash(const Graph* g, hipStream_t s, uint64_t* out) {
  const size_t total = (size_t)g->ndir * g->N * sizeof(double);
  const size_t chunk = size_t(16) << 20;
  std::vector<unsigned char> buf(std::min(total, chunk));
  uint64_t h = 1469598103934665603ull;
  for (size_t off = 0; off < total; off += chunk) {
    const size_t n = std::min(chunk, total - off);
    RW_HIP(hipMemcpyAsync(buf.data(), reinterpret_cast<const char*>(g->weight) + off, n, hipMemcpyDeviceToHost, s));
    RW_HIP(hipStreamSynchronize(s));
    for (size_t k = 0; k < n; ++k) {
      h ^= buf[k];
      h *= 1099511628211ull;
    }
  }
  *out = h;
  return RW_OK;
}

static int read_header(FILE* f, const char* path, rw_eig_header* hdr) {
  RW_CHECK(fread(hdr, sizeof(*hdr), 1, f) == 1, RW_EINVAL, "%s: shorter than a checkpoint header", path);
  RW_CHECK(std::memcmp(hdr->magic, kMagic, sizeof(kMagic)) == 0, RW_EINVAL, "%s: not an eigenpair checkpoint",
           path);
  RW_CHECK(hdr->version == 1, RW_EINVAL, "%s: checkpoint version %d is not supported", path, hdr->version);
  RW_CHECK(hdr->m >= 1 && q_dtype_ok(hdr->q_dtype) &&
               hdr->dims[0] >= 1 && hdr->dims[1] >= 1 && hdr->dims[2] >= 1,
           RW_EINVAL, "%s: corrupt checkpoint header", path);
  const uint64_t N = (uint64_t)hdr->dims[0] * hdr->dims[1] * hdr->dims[2];
  RW_CHECK(hdr->q_bytes == N * q_block_cols(hdr->q_dtype, hdr->m) * dtype_size(hdr->q_dtype) &&
               hdr->lambda_bytes == (uint64_t)hdr->m * 8,
           RW_EINVAL, "%s: corrupt checkpoint header (sizes)", path);
  return RW_OK;
}

struct FileCloser {
  FILE* f;
  ~FileCloser() {
    if (f) fclose(f);
  }
};

}  // namespace rw

using namespace rw;

extern "C" {

int rw_eig_save(rw_graph h, const char* path, const void* Q, int q_dtype, const double* lambda, int m, double tol,
                hipStream_t stream) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr && path != nullptr && Q != nullptr && lambda != nullptr, RW_EINVAL, "null argument");
  RW_CHECK(q_dtype_ok(q_dtype), RW_EINVAL, "bad Q dtype");
  const Graph* g = &h->g;
  RW_CHECK(m >= 1 && m <= g->N, RW_EINVAL, "m = %d out of range", m);
  rw_eig_header hdr;
  std::memset(&hdr, 0, sizeof(hdr));
  std::memcpy(hdr.magic, kMagic, sizeof(kMagic));
  hdr.version = 1;
  hdr.ndim = g->ndim;
  hdr.conn = g->conn;
  hdr.graph_dtype = g->dtype;
  hdr.weight_form = g->weight_form;
  hdr.normalized = g->normalized;
  hdr.dims[0] = g->nx;
  hdr.dims[1] = g->ny;
  hdr.dims[2] = g->nz;
  hdr.beta = g->beta;
  hdr.m = m;
  hdr.q_dtype = q_dtype;
  hdr.tol = tol;
  RW_TRY(weight_hash(g, stream, &hdr.weight_hash));
  hdr.q_bytes = (uint64_t)g->N * q_block_cols(q_dtype, m) * dtype_size(q_dtype);
  hdr.lambda_bytes = (uint64_t)m * 8;
  FileCloser fc{fopen(path, "wb")};
  RW_CHECK(fc.f != nullptr, RW_EINVAL, "cannot open %s for writing", path);
  RW_CHECK(fwrite(&hdr, sizeof(hdr), 1, fc.f) == 1, RW_EINVAL, "%s: write failed", path);
  const size_t chunk = size_t(64) << 20;
  std::vector<char> buf(std::min<size_t>(hdr.q_bytes, chunk));
  for (uint64_t off = 0; off < hdr.q_bytes; off += chunk) {
    const size_t n = (size_t)std::min<uint64_t>(chunk, hdr.q_bytes - off);
    RW_HIP(hipMemcpyAsync(buf.data(), static_cast<const char*>(Q) + off, n, hipMemcpyDeviceToHost, stream));
    RW_HIP(hipStreamSynchronize(stream));
    RW_CHECK(fwrite(buf.data(), 1, n, fc.f) == n, RW_EINVAL, "%s: write failed", path);
  }
  std::vector<double> lam((size_t)m);
  RW_HIP(hipMemcpyAsync(lam.data(), lambda, hdr.lambda_bytes, hipMemcpyDeviceToHost, stream));
  RW_HIP(hipStreamSynchronize(stream));
  RW_CHECK(fwrite(lam.data(), 8, (size_t)m, fc.f) == (size_t)m, RW_EINVAL, "%s: write failed", path);
  RW_CHECK(fflush(fc.f) == 0, RW_EINVAL, "%s: write failed", path);
  return RW_OK;
}

int rw_eig_read_header(const char* path, rw_eig_header* hdr) {
  RW_CHECK(path != nullptr && hdr != nullptr, RW_EINVAL, "null argument");
  FileCloser fc{fopen(path, "rb")};
  RW_CHECK(fc.f != nullptr, RW_EINVAL, "cannot open %s", path);
  return read_header(fc.f, path, hdr);
}

int rw_eig_load(rw_graph h, const char* path, void* Q, int q_dtype, double* lambda, int m, hipStream_t stream,
                rw_eig_header* out_hdr) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr && path != nullptr && Q != nullptr && lambda != nullptr, RW_EINVAL, "null argument");
  const Graph* g = &h->g;
  FileCloser fc{fopen(path, "rb")};
  RW_CHECK(fc.f != nullptr, RW_EINVAL, "cannot open %s", path);
  rw_eig_header hdr;
  RW_TRY(read_header(fc.f, path, &hdr));
  RW_CHECK(hdr.ndim == g->ndim && hdr.conn == g->conn && hdr.dims[0] == g->nx && hdr.dims[1] == g->ny &&
               hdr.dims[2] == g->nz,
           RW_EINVAL, "%s: computed for a %lld x %lld x %lld grid (connectivity %d), not this graph", path,
           (long long)hdr.dims[0], (long long)hdr.dims[1], (long long)hdr.dims[2], hdr.conn);
  RW_CHECK(hdr.normalized == g->normalized && hdr.weight_form == g->weight_form, RW_EINVAL,
           "%s: computed for another operator form (normalized %d, weight form %d)", path, hdr.normalized,
           hdr.weight_form);
  RW_CHECK(q_dtype == hdr.q_dtype, RW_EINVAL, "%s: holds Q of dtype %d, not %d", path, hdr.q_dtype, q_dtype);
  RW_CHECK(m >= 1 && m <= hdr.m, RW_EINVAL, "%s: holds %d pairs, %d requested", path, hdr.m, m);
  uint64_t hash = 0;
  RW_TRY(weight_hash(g, stream, &hash));
  RW_CHECK(hash == hdr.weight_hash, RW_EINVAL,
           "%s: computed for other edge weights (beta %.17g then; the graph was built or edited since)", path,
           hdr.beta);
  // the first m pairs are a prefix of the stored block (the pair form's remainder columns come first);
  // lambda follows the whole block
  const size_t es = dtype_size(q_dtype);
  const uint64_t want = (uint64_t)g->N * q_block_cols(q_dtype, m) * es;
  const size_t chunk = size_t(64) << 20;
  std::vector<char> buf(std::min<size_t>(want, chunk));
  for (uint64_t off = 0; off < want; off += chunk) {
    const size_t n = (size_t)std::min<uint64_t>(chunk, want - off);
    RW_CHECK(fread(buf.data(), 1, n, fc.f) == n, RW_EINVAL, "%s: truncated", path);
    RW_HIP(hipMemcpyAsync(static_cast<char*>(Q) + off, buf.data(), n, hipMemcpyHostToDevice, stream));
    RW_HIP(hipStreamSynchronize(stream));
  }
  RW_CHECK(fseeko(fc.f, (off_t)(sizeof(hdr) + hdr.q_bytes), SEEK_SET) == 0, RW_EINVAL, "%s: truncated", path);
  std::vector<double> lam((size_t)hdr.m);
  RW_CHECK(fread(lam.data(), 8, (size_t)hdr.m, fc.f) == (size_t)hdr.m, RW_EINVAL, "%s: truncated", path);
  RW_HIP(hipMemcpyAsync(lambda, lam.data(), (size_t)m * 8, hipMemcpyHostToDevice, stream));
  RW_HIP(hipStreamSynchronize(stream));
  if (out_hdr) *out_hdr = hdr;
  return RW_OK;
}

}  // extern "C"
