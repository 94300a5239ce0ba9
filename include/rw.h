/*
 * rw.h - C ABI of librw, a gfx950 (MI355X) implementation of precomputed-eigenvector random-walker
 * segmentation (Andrews & Hamarneh, "Adaptable Precomputation for Random Walker Image Segmentation
 * and Registration").
 *
 * Conventions (every entry point):
 *   - Returns an int status: RW_OK (0) or a negative RW_E* code.  No exception or abort crosses the
 *     ABI.  rw_last_error() returns a message for the calling thread's last failure.
 *   - All device memory is owned by the caller: inputs, outputs, the graph buffer and workspaces
 *     are device pointers the caller allocated (sizes from the *_bytes / *_workspace_bytes queries).
 *     The library never allocates device memory.  Host arrays (seeds, edit lists) are read during
 *     the call and not retained.
 *   - Work is enqueued on the given HIP stream.  Calls that must inspect a device result (a status
 *     word, a convergence test) synchronize that stream before returning; all others return after
 *     enqueueing.
 *   - Images have dims (nx, ny, nz) (nz = 1 in 2D) and N = nx*ny*nz nodes numbered
 *     i = x + nx*(y + ny*z).  Blocks of vectors are column-major N x b: vector j occupies
 *     [j*N, (j+1)*N).  Label maps are C x N (label k's map contiguous).
 *   - Edges are numbered e = dir*N + tail for the edge joining `tail` and tail + offset(dir), with
 *     forward directions in this order: 2D 4-connected (+x, +y); 2D 8-connected (+x, +y, +x+y, +x-y);
 *     3D 6-connected (+x, +y, +z).  An id whose head lies outside the grid is invalid.
 */
#ifndef RW_H
#define RW_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define RW_OK 0
#define RW_EINVAL (-1)       /* an argument is out of range or inconsistent */
#define RW_ENOCONV (-2)      /* an iteration hit its limit; the best iterate is left in the outputs */
#define RW_EUNANCHORED (-3)  /* a connected component of the graph holds no seed (gamma = 0) */
#define RW_ESINGULAR (-4)    /* a small dense system has a pivot below its threshold */
#define RW_EWORKSPACE (-5)   /* the buffer passed is smaller than the query returned */
#define RW_EHIP (-6)         /* a HIP runtime call failed */
#define RW_ECAPTURE (-7)     /* a synchronous call on a stream under HIP graph capture (nothing was enqueued) */

/* ---- element types ---- */
#define RW_F64 0
#define RW_F32 1
#define RW_BF16 2
/* BF16 pair form of an eigenbasis (rw_convert_block, rw_solve_seeds*, checkpoints): a column-major
 * N x (RW_PAIR_COLS + m) BF16 block whose first RW_PAIR_COLS columns hold the rounding remainders
 * bf16(q_j - bf16(q_j)) of columns j = 1 .. RW_PAIR_COLS (zero where j >= m) and whose last m columns are
 * the plain BF16 copy bf16(q_j), j = 0 .. m-1.  Column j <= RW_PAIR_COLS is read as hi + lo (about 16
 * significant bits); the others as BF16.  The low-index columns carry the largest coefficients of the
 * online solve, so the remainder columns remove most of the BF16 rounding error of the maps for 8 extra
 * columns of traffic.  The plain BF16 block starts at column RW_PAIR_COLS. */
#define RW_BF16_PAIR 3
#define RW_PAIR_COLS 8

/* ---- edge-weight forms (Sec. II-A, eq. (2)) ---- */
#define RW_WEIGHT_SQUARED 0  /* w = s_e * exp(-beta (J_i - J_j)^2) (default) */
#define RW_WEIGHT_ABS 1      /* w = s_e * exp(-beta |J_i - J_j|)   (the paper's printed form) */

typedef struct rw_graph_s* rw_graph;

typedef struct {
  int32_t ndim;        /* 2 or 3 */
  int64_t dims[3];     /* nx, ny, nz; nz = 1 when ndim = 2; each >= 1, N >= 2 */
  int32_t conn;        /* 4 or 8 when ndim = 2; 6 when ndim = 3 */
  int32_t dtype;       /* RW_F64 or RW_F32: type of the operator's stored coefficients (coef, diag, dinv,
                          ghat) and of rw_apply_laplacian; scales, weights and degrees are FP64 always */
  int32_t weight_form; /* RW_WEIGHT_SQUARED or RW_WEIGHT_ABS */
  int32_t normalized;  /* 1: the operator is L_hat = D^{-1/2} L D^{-1/2} (Sec. II-C); 0: L = D - W */
} rw_graph_desc;

const char* rw_last_error(void);
int rw_version(void);

/* ======================================================================================
 * Graph (Sec. II-A eq. (2); Sec. II-C)
 * ====================================================================================== */

/* Bytes of device memory rw_build_graph needs for this description. */
int rw_graph_bytes(const rw_graph_desc* desc, size_t* bytes);

/* Build the weighted image graph of intensities J (device, N values of J_dtype = RW_F64 or RW_F32)
 * with parameter beta >= 0 into the caller's device buffer graph_buf (>= rw_graph_bytes; it must
 * stay allocated while the handle is used; J is copied).  Computes per forward edge the weight, a
 * presence bit (uint8 mask per node, bit dir), the degree d, d^{-1/2} (0 where d = 0), the unit null
 * vector (D^{1/2}1/||D^{1/2}1|| or 1/sqrt(N)) and the operator's coefficients.  Every edge starts
 * present with scale 1.  *out receives a host handle; free it with rw_graph_destroy.
 * Errors: RW_EINVAL (bad description, beta < 0 or not finite, null pointers), RW_EWORKSPACE. */
int rw_build_graph(const rw_graph_desc* desc, const void* J_dev, int J_dtype, double beta,
                   void* graph_buf, size_t buf_bytes, hipStream_t stream, rw_graph* out);

int rw_graph_destroy(rw_graph g);

/* Device views of the graph's arrays (for tests and for callers that fuse their own work).
 * coef, diag, dinv and ghat are of the graph's dtype; J, weight, scale and degree are FP64 on every
 * graph (an FP32 graph rounds only the operator's coefficients, once, from the FP64 values).  Planes
 * are ndir x N, direction-major. */
typedef struct {
  int64_t N;
  int32_t ndir;
  int32_t dtype;
  double beta;
  const double* J;      /* N, FP64 copy of the intensities */
  const double* weight; /* ndir x N: w_e = s_e * exp(...) in FP64 (0 where absent / off-grid) */
  const double* scale;  /* ndir x N: s_e in FP64 (0 where absent / off-grid) */
  const void* coef;     /* ndir x N: off-diagonal magnitude of the operator, w_e d_i^{-1/2} d_j^{-1/2} or w_e */
  const void* diag;     /* N: diagonal of the operator (1 or 0 for L_hat, d for L) */
  const void* dinv;     /* N: d^{-1/2} (0 where d = 0) */
  const void* ghat;     /* N: unit null vector */
  const double* degree; /* N: d in FP64 */
  const uint8_t* mask;  /* N: bit dir set iff the forward edge in direction dir is present */
  const int64_t* comp;  /* N: component root (smallest node index) over edges with w >= 1e-30; valid after
                           rw_graph_components (or any solve) since the last build or edit */
} rw_graph_view;
int rw_graph_get_view(rw_graph g, rw_graph_view* view);

/* Connected components of the graph restricted to edges with w >= 1e-30, the topology on which the
 * gamma = 0 systems of eq. (5) and of the eigenbasis solve are solvable: a component without a seed makes
 * them singular, and rw_solve_seeds / rw_cg_solve / rw_cg_solve_rhs then fail with RW_EUNANCHORED.
 * Computed on the device (hooking and pointer jumping) on first use after a build or edit and cached;
 * n_components (host, may be null) receives their number.  Synchronizes `stream`. */
int rw_graph_components(rw_graph g, int64_t* n_components, hipStream_t stream);

/* Edits of the graph, applied in array order (Sec. III-B changes beta; the others are weight and
 * topology edits).  Edge ids must be valid and present (else RW_EINVAL, nothing applied).
 * SET_BETA recomputes every weight from J with the new beta and keeps the edge scales;
 * SCALE_EDGES / SCALE_BOX multiply the scale of the listed edges / of the present edges with both
 * endpoints inside [box_lo, box_hi) by `value` (> 0); REMOVE_EDGES sets their scale to 0 and clears
 * their mask bits.  Degrees, d^{-1/2}, the null vector and the operator are rebuilt afterwards. */
#define RW_EDIT_SET_BETA 0
#define RW_EDIT_SCALE_EDGES 1
#define RW_EDIT_SCALE_BOX 2
#define RW_EDIT_REMOVE_EDGES 3
typedef struct {
  int32_t kind;
  double value;              /* new beta, or the scale factor */
  const int64_t* edge_ids;   /* host array of n edge ids (SCALE_EDGES, REMOVE_EDGES) */
  int64_t n;
  int64_t box_lo[3];         /* SCALE_BOX: inclusive lower corner (x, y, z) */
  int64_t box_hi[3];         /* SCALE_BOX: exclusive upper corner */
} rw_edit;
int rw_edit_graph(rw_graph g, const rw_edit* edits, int n_edits, hipStream_t stream);

/* ======================================================================================
 * Stencil operator (Sec. II-A: L = D - W; Sec. II-C: L_hat)
 * ====================================================================================== */

/* Y = op(X) for a column-major N x b block in the graph's dtype (X, Y distinct device buffers),
 * op = L_hat or L per the graph description.  Matrix-free over the 4/8/6-point stencil. */
int rw_apply_laplacian(rw_graph g, const void* X, void* Y, int64_t b, hipStream_t stream);

/* Fused form used by polynomial filters: Y = alpha * op(X) + beta * X + gamma * Z (Z may be null
 * when gamma = 0; Z may alias Y). */
int rw_apply_laplacian_axpby(rw_graph g, const void* X, void* Y, const void* Z, int64_t b,
                             double alpha, double beta, double gamma, hipStream_t stream);

/* rw_apply_laplacian for b >= 1 with its one operator kernel launched through hipExtLaunchKernel, so that
 * `start` and `stop` (events the caller created with timing enabled on the stream's device) record that
 * dispatch's own start and end: hipEventElapsedTime(start, stop) is the kernel's duration as a kernel
 * trace reports it, without the stream's progress around the launch.  A measurement hook: the result is
 * bit-identical to rw_apply_laplacian's.  RW_EINVAL for a null event or b < 1, RW_EHIP when the launch
 * fails. */
int rw_apply_laplacian_timed(rw_graph g, const void* X, void* Y, int64_t b, hipStream_t stream,
                             hipEvent_t start, hipEvent_t stop);

/* ======================================================================================
 * Offline eigenpairs (Sec. II-B eq. (6): the m smallest eigenpairs, null pair included)
 * ====================================================================================== */
typedef struct {
  double tol;        /* stop when ||op q_i - lambda_i q_i|| <= tol for every returned pair */
  int32_t max_iter;  /* outer (filter + Rayleigh-Ritz) iterations */
  int32_t degree;    /* Chebyshev filter degree per outer iteration (0 -> library default) */
  int32_t guard;     /* block columns beyond m (0 -> max(8, ceil(m/10))) */
  uint64_t seed;     /* seed of the random start block */
  int32_t warm;      /* 1: start from the columns already in Q (m of them) */
  int32_t q_dtype;   /* RW_F64 or RW_F32: storage of Q and of the block iteration */
} rw_eig_opts;

typedef struct {
  int32_t iters;        /* outer iterations run */
  int32_t n_converged;  /* pairs meeting tol */
  int64_t spmm_columns; /* total columns passed through the stencil operator */
  double max_residual;  /* max_i ||op q_i - lambda_i q_i|| */
  double seconds;       /* wall time of the call */
} rw_eig_info;

int rw_eig_workspace_bytes(rw_graph g, int m, const rw_eig_opts* opts, size_t* bytes);

/* Compute the m smallest eigenpairs of the graph operator into Q (device, column-major N x m of
 * opts->q_dtype) and lambda (device, m FP64, increasing).  Column 0 is the analytic unit null
 * vector with lambda = 0; columns 1.. are orthonormal and orthogonal to it.
 * Errors: RW_EINVAL (m < 2 or m + guard > N - 1, bad opts), RW_EWORKSPACE, RW_ENOCONV (the best
 * iterate is left in Q, lambda). */
int rw_precompute_eig(rw_graph g, int m, const rw_eig_opts* opts, void* Q, double* lambda, void* work,
                      size_t work_bytes, hipStream_t stream, rw_eig_info* info);

/* ======================================================================================
 * Online update after graph edits (Sec. III-B)
 * ====================================================================================== */
#define RW_UPDATE_DIAG_RQ 0 /* the paper: Q kept (null vector replaced, re-orthonormalized in order),
                                lambda_i <- q_i^T op_new q_i (eqs. (26)-(28)) */
#define RW_UPDATE_RR 1      /* Rayleigh-Ritz of op_new on the same span: Q <- Q V, lambda <- Ritz values */
#define RW_UPDATE_RR_REFINE 2 /* RR, then filtered subspace iterations warm-started from Q until
                                 the residuals are <= opts->tol */

int rw_update_workspace_bytes(rw_graph g, int m, const rw_eig_opts* opts, size_t* bytes);

/* Apply the edits to the graph (as rw_edit_graph), then update the stored pairs (Q, lambda) of m
 * columns (Q of opts->q_dtype) for the new operator by `mode`.
 * Errors: RW_EINVAL, RW_EWORKSPACE, RW_ENOCONV (mode 2). */
int rw_update_eig(rw_graph g, const rw_edit* edits, int n_edits, int mode, const rw_eig_opts* opts,
                  void* Q, double* lambda, int m, void* work, size_t work_bytes, hipStream_t stream,
                  rw_eig_info* info);

/* Bank of bases precomputed for several beta (Sec. III-B, last paragraph: eigenvectors for several beta, with
 * the Rayleigh quotients of eq. (26) interpolating between them).  For g's current operator, every basis of the
 * bank (nbank device pointers, each column-major N x m of opts->q_dtype, the graph's dtype) gets the diagonal
 * update of rw_update_eig's RW_UPDATE_DIAG_RQ mode (eq. (27): null vector replaced, the other columns
 * re-orthonormalized in order, lambda_hat_i = q_i^T op q_i), and the basis whose quotients sum lowest is
 * written, updated, to Q_out (device, N x m, not a bank basis) with lambda_out (device, m FP64).  The smallest
 * sum marks the basis closest to the current low spectrum: the eigenbasis of the m smallest eigenvalues has
 * the smallest sum among orthonormal bases (Ky Fan).  The bank is read only.  *chosen (host) receives the
 * index; traces (host, nbank, may be null) the sums.  work: rw_bank_workspace_bytes.  Synchronizes `stream`.
 * Errors: RW_EINVAL, RW_EWORKSPACE, RW_ESINGULAR (a basis is linearly dependent). */
int rw_bank_workspace_bytes(rw_graph g, int m, const rw_eig_opts* opts, size_t* bytes);
int rw_bank_select(rw_graph g, const void* const* Q_bank, int nbank, const rw_eig_opts* opts, int m, void* Q_out,
                   double* lambda_out, void* work, size_t work_bytes, hipStream_t stream, int* chosen,
                   double* traces);

/* ---- vertex aggregation (Sec. III-C) over regular blocks of s x s (x s) voxels, the last ones clipped ---- */

/* Description of the aggregated graph of g for blocks of s (the block grid, g's connectivity, dtype, weight form
 * and operator form).  Host only.  Errors: RW_EINVAL (s < 1, fewer than two blocks). */
int rw_aggregate_desc(rw_graph g, int s, rw_graph_desc* desc);
int rw_aggregate_workspace_bytes(rw_graph g, int s, size_t* bytes);
/* Build the aggregated graph in coarse_buf (rw_graph_bytes of rw_aggregate_desc): intensities 0 and per-edge
 * scales equal to the summed FP64 weights of g's edges joining the two blocks, so its Laplacian is P^T L P for
 * the 0/1 assignment matrix P.  The caller destroys it with rw_graph_destroy.  Synchronizes `stream`. */
int rw_aggregate_graph(rw_graph g, int s, void* coarse_buf, size_t coarse_bytes, void* work, size_t work_bytes,
                       hipStream_t stream, rw_graph* coarse);
/* Eq. (33): Qc(y, j) = sum over the vertices x of block y of Delta(x) Q(x, j) / |y|, with Delta(x) twice the
 * number of x's present edges whose other end lies in another block (the edges inside a block are consumed by
 * it).  Q device column-major N x m (RW_F64 or RW_F32), Qc device N_bar x m of the same type.  Follow with
 * rw_update_eig(coarse, NULL, 0, RW_UPDATE_DIAG_RQ, ...) for the Gram-Schmidt step and the normalized-cut values
 * on the aggregated graph. */
int rw_aggregate_basis(rw_graph g, int s, const void* Q, int q_dtype, int m, void* Qc, void* work,
                       size_t work_bytes, hipStream_t stream);
/* Seeds moved to their blocks (host arrays; out_* hold at least S entries): sorted, distinct.  Errors: RW_EINVAL
 * (a node out of range, two labels in one block). */
int rw_aggregate_seeds(rw_graph g, int s, const int64_t* seed_node, const int32_t* seed_label, int64_t S,
                       int64_t* out_node, int32_t* out_label, int64_t* S_out);
/* Propagation back to g (eq. (30) with eta(x, y) = 1 for x's block): U(c, x) = Uc(c, block of x); Uc device
 * C x N_bar, U device C x N, g's dtype. */
int rw_prolong(rw_graph g, int s, const void* Uc, int C, void* U, hipStream_t stream);

/* ======================================================================================
 * Checkpoint of the offline phase (Sec. II-B: the eigenpairs are computed once, offline)
 * ====================================================================================== */
typedef struct {
  char magic[8];          /* "RWEIGv1" */
  int32_t version;        /* 1 */
  int32_t ndim, conn, graph_dtype, weight_form, normalized;
  int64_t dims[3];
  double beta;            /* beta of the graph when saved */
  int32_t m, q_dtype;     /* pairs stored, storage type of Q */
  double tol;             /* residual tolerance the pairs were computed to (as given by the caller) */
  uint64_t weight_hash;   /* 64-bit FNV-1a of the FP64 edge weights (ndir x N, 0 where absent) */
  uint64_t q_bytes, lambda_bytes;
  int32_t reserved[6];    /* zero */
} rw_eig_header;

/* Write the eigenpairs (Q: device, column-major N x m of q_dtype, or the N x (RW_PAIR_COLS + m) pair form;
 * lambda: device, m FP64) of graph g to
 * the file `path` (created or truncated): the header above, then Q's bytes, then lambda's.  The weight
 * hash ties the file to g's current operator.  Synchronizes `stream`.  Errors: RW_EINVAL (bad argument,
 * the file cannot be written), RW_EHIP. */
int rw_eig_save(rw_graph g, const char* path, const void* Q, int q_dtype, const double* lambda, int m,
                double tol, hipStream_t stream);
/* Read and validate a checkpoint's header (host only, no device work).  Errors: RW_EINVAL (cannot open,
 * not a checkpoint, unsupported version, inconsistent sizes). */
int rw_eig_read_header(const char* path, rw_eig_header* hdr);
/* Load the first m (<= stored) pairs of a checkpoint into Q (device, N x m of q_dtype, or the pair form's
 * N x (RW_PAIR_COLS + m); q_dtype must equal the
 * stored type) and lambda (device, m FP64), after checking that the file was written for this grid,
 * connectivity and operator form and that the hash of g's current edge weights equals the stored one (a
 * graph built with another beta, or edited since, is refused).  hdr (host, may be null) receives the
 * header.  Synchronizes `stream`.  Errors: RW_EINVAL (any mismatch, truncated file), RW_EHIP. */
int rw_eig_load(rw_graph g, const char* path, void* Q, int q_dtype, double* lambda, int m, hipStream_t stream,
                rw_eig_header* hdr);

/* ======================================================================================
 * Online random-walker solve in the eigenbasis (Sec. II-B eqs. (7)-(17), gamma = 0 case after
 * eq. (17); choice of m, Sec. III-A1 eq. (24))
 * ====================================================================================== */
typedef struct {
  int32_t m_used;    /* eigenpairs used */
  double f_max;      /* S * eps^2 (0 when eps <= 0) */
  double f_worst;    /* max over labels of the fit (eq. (24)) at m_used (0 when eps <= 0) */
  double min_pivot;  /* smallest |pivot| / max|entry| of the reduced system's LU */
  int32_t eig_probes; /* choice of m: batched eigen-based evaluations the Cholesky screen left (0 when eps <= 0) */
} rw_solve_info;

int rw_solve_workspace_bytes(rw_graph g, int m_avail, int64_t S, int C, size_t* bytes);

/* Label probabilities of the gamma = 0 random walker from the stored pairs (Q, lambda):
 *   Q        device, column-major N x (>= m_avail) of q_dtype (RW_F64, RW_F32 or RW_BF16), or the
 *            N x (RW_PAIR_COLS + (>= m_avail)) BF16 pair form (q_dtype RW_BF16_PAIR), with
 *            column 0 the graph's unit null vector and the other columns orthogonal to it (as
 *            rw_precompute_eig / rw_update_eig return them); lambda device FP64, lambda[0] = 0;
 *   seeds    host arrays seed_node[S] (0 <= node < N) and seed_label[S] (0 <= label < C); any order;
 *            a repeated node with the same label counts once, with different labels is RW_EINVAL;
 *   eps      <= 0: use m = m_avail; > 0: m = the smallest m in [2, m_avail] whose fit of every
 *            label's seeds (eq. (24), rho = sqrt(1^T D 1) or sqrt(N)) is <= S * eps^2;
 *   U        device C x N of the graph's dtype; seed rows are one-hot, a label without seeds is 0.
 * Seeds are sorted ascending.  After m is chosen (the fit uses the stored columns), the basis is taken
 * in FP64 as Q' = [g, (q_j - g c_j) / n_j], with g the graph's exact FP64 null vector, c_j = g^T q_j and
 * n_j the norm (one pass over Q's first m columns), and the reduced (m x m) system
 *   (Lambda - Q'_s^T B Q'_n) Y = Q'_s^T op_ss U_hat_s
 * is formed from the FP64 weights and degrees and solved (FP64 LU with partial pivoting);
 * U_hat_n = Q'_n Y, U = D^{-1/2} U_hat on non-seeds.  This system is algebraically the (S+1) x (S+1)
 * bordered seed system of the paper's gamma = 0 case with F_s eliminated.  The call synchronizes `stream`.
 * Errors: RW_EINVAL (also: a column of Q in the span of column 0), RW_EWORKSPACE, RW_EUNANCHORED (a
 * component of the anchoring graph holds no seed), RW_ESINGULAR (pivot < 1e-14 * max|entry|); U is not
 * valid when the call fails. */
int rw_solve_seeds(rw_graph g, const void* Q, int q_dtype, const double* lambda, int m_avail,
                   const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C, double eps,
                   void* U, void* work, size_t work_bytes, hipStream_t stream, rw_solve_info* info);

/* ---- gamma > 0: prior probabilities (Sec. II-A eq. (5); Sec. II-B eqs. (15), (17); Sec. III-A2 eq. (25)) ---- */

int rw_solve_prior_workspace_bytes(rw_graph g, int m_avail, int64_t S, int C, size_t* bytes);

/* Label probabilities of the random walker with priors P and weight gamma > 0 from the stored pairs:
 * (L_n + gamma I) U_n = gamma P_n - B^T U_s in the variables of the graph's operator (under the normalized
 * Laplacian the prior enters as P_hat = D^{1/2} P, so U solves (L_n + gamma D_n) U_n = gamma D_n P_n -
 * B^T U_s).  With E = Q (Lambda + gamma I)^{-1} Q^T, eq. (17) for F_s and eq. (15) for U_n are evaluated in
 * their m x m reduced form: with G = B Q'_n, Z = Q'_n^T P_hat_n and Lambda_g = Lambda + gamma I,
 *   (Lambda_g - Q'_s^T G) V = Q'_s^T [op_ss U_hat_s + gamma (U_hat_s + G Lambda_g^{-1} Z)],
 *   U_hat_n = Q'_n (V + gamma Lambda_g^{-1} Z),
 * on the FP64 basis Q' of rw_solve_seeds (FP64 LU with partial pivoting).  No seed needs to reach every
 * component (L_n + gamma I is definite).
 *   Q, q_dtype, lambda, m_avail, seeds, C, U, work: as rw_solve_seeds (work: rw_solve_prior_workspace_bytes);
 *   prior    device C x N (label k's map contiguous) of prior_dtype (RW_F64 or RW_F32), read-only;
 *   gamma    > 0;
 *   eps      <= 0: m = m_avail; > 0: m = the smallest m in [2, m_avail] with g_k(m) = ||p_k - Q_m Q_m^T p_k||^2
 *            <= g_max = eps^2 n for the sampled labels k = 0, r^d, 2 r^d, ... (d the image dimension), with
 *            p = P_hat and n = 1^T D 1 under the normalized Laplacian (p = P, n = N under L); g_k is taken
 *            from one projection of P_hat on the stored columns (Q orthonormal: g_k(m) = ||p_k||^2 minus the
 *            first m squared coefficients), m_avail when no m qualifies;
 *   info     m_used, f_max = g_max, f_worst = max over the sampled labels of g_k(m_used) (0 when eps <= 0),
 *            min_pivot.
 * The call synchronizes `stream`.  Errors: RW_EINVAL, RW_EWORKSPACE, RW_ESINGULAR. */
int rw_solve_seeds_prior(rw_graph g, const void* Q, int q_dtype, const double* lambda, int m_avail,
                         const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C, double gamma,
                         const void* prior, int prior_dtype, double eps, int r, void* U, void* work,
                         size_t work_bytes, hipStream_t stream, rw_solve_info* info);

/* Workspace of rw_solve_priors for these sizes (labels != 0 when the call asks for labels). */
int rw_solve_priors_workspace_bytes(rw_graph g, int q_dtype, int m_avail, int C, int r, int labels,
                                    size_t* bytes);

/* The walker driven by priors alone, at registration label counts (thousands of displacement labels):
 * eq. (5) of Sec. II-A with the seed set empty, (L + gamma I) U = gamma P on every vertex, in the variables of
 * the graph's operator (under the normalized Laplacian (L_hat + gamma I) U_hat = gamma P_hat, i.e.
 * (L + gamma D) U = gamma D P), approximated in the eigenbasis by eq. (15) of Sec. II-B with no seed rows:
 *   U_hat = Q' (Lambda + gamma I)^{-1} gamma Q'^T P_hat,
 * on the FP64 basis Q' of rw_solve_seeds (the exact null vector first, the other columns made orthogonal to it).
 * Registration's result is, at each voxel, the label of largest probability (its displacement).
 *   Q, q_dtype  device m_avail x N basis: RW_F64, RW_F32 or RW_BF16 (column 0 the null pair's); with RW_BF16
 *            the projection and the labels run on the matrix cores (FP32 accumulation; m_avail <= 223);
 *   lambda   device m_avail eigenvalues (FP64);
 *   prior    device C x N (label k's map contiguous), RW_BF16 or RW_F32 with a BF16 basis, RW_F64 or RW_F32
 *            otherwise; read-only;
 *   gamma    > 0;
 *   eps, r   eps <= 0: m = m_avail; > 0: the choice of m of rw_solve_seeds_prior (eq. (25) on the labels 0,
 *            r^d, 2 r^d, ..., d the image dimension);
 *   U        device C x N of the graph's dtype, or null: the probabilities;
 *   label, prob  device N int32 and N of the graph's dtype, or both null: per voxel the smallest label of
 *            largest probability and that probability (label 0, probability 0 on a vertex of degree 0);
 *            with a BF16 basis evaluated by the fused reconstruction (U not formed), otherwise with the same
 *            arithmetic as U;
 *   work     rw_solve_priors_workspace_bytes(g, q_dtype, m_avail, C, r, label != null) bytes of device memory;
 *   info     m_used, f_max = g_max and f_worst = the largest sampled g_k(m_used) (0 when eps <= 0).
 * At least one of U and label must be asked for.  The call synchronizes `stream`.  Errors: RW_EINVAL (also: a
 * basis column in the null vector's span), RW_EWORKSPACE, RW_ECAPTURE. */
int rw_solve_priors(rw_graph g, const void* Q, int q_dtype, const double* lambda, int m_avail, const void* prior,
                    int prior_dtype, int C, double gamma, double eps, int r, void* U, int32_t* label, void* prob,
                    void* work, size_t work_bytes, hipStream_t stream, rw_solve_info* info);

int rw_priors_workspace_bytes(int C, size_t* bytes);

/* Prior probabilities from the seeds (Sec. IV-A): per label, a Gaussian fitted to the intensities J of its
 * seeds (mean and maximum-likelihood variance, FP64, floored at 1e-6); prior(k, i) = that density at J_i
 * normalized over the labels that have seeds (a softmax of the log-densities); a label without seeds gets 0.
 * seed_node, seed_label: device arrays of S entries (any order); prior: device C x N of prior_dtype (RW_F64 or
 * RW_F32); work: rw_priors_workspace_bytes(C); *status (device int32) receives RW_OK, or RW_EINVAL when a
 * seed is out of range (such seeds are skipped).  Only enqueues kernels (capturable).  Errors of the call:
 * RW_EINVAL, RW_EWORKSPACE. */
int rw_priors_from_seeds(rw_graph g, const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C,
                         void* prior, int prior_dtype, void* work, size_t work_bytes, int32_t* status,
                         hipStream_t stream);

/* RW_ASYNC form of rw_solve_seeds, for streams under HIP graph capture and callers that must not wait:
 * it only enqueues kernels (no host read, no wait, no memset) and reports through *status (device int32):
 * RW_OK, or RW_EINVAL (a seed or label out of range, seeds not strictly ascending, a basis column in the
 * null vector's span), RW_EUNANCHORED or RW_ESINGULAR as rw_solve_seeds would; U is valid only when it is
 * RW_OK.  Differences from rw_solve_seeds: the seeds are device arrays (seed_node ascending and distinct,
 * seed_label in [0, C)), m is fixed (no choice of m), and the graph's components must be current
 * (rw_graph_components after the last build or edit; the call fails with RW_EINVAL otherwise).  work:
 * at least rw_solve_workspace_bytes(g, m, S, C) bytes.  The same kernels as rw_solve_seeds with eps <= 0 and
 * m_avail = m give the same results.  A captured graph of this call stays valid while the graph, Q, lambda,
 * the buffers and S, C and m stay the same; the seed arrays' contents may change between replays.
 * Errors returned by the call itself (nothing enqueued): RW_EINVAL, RW_EWORKSPACE. */
int rw_solve_seeds_async(rw_graph g, const void* Q, int q_dtype, const double* lambda, int m,
                         const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C, void* U,
                         void* work, size_t work_bytes, int32_t* status, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): rw_solve_seeds with a fixed m (no choice of m; same kernels, same results as
 * rw_solve_seeds with eps <= 0 and m_avail = m) that calls no hipMalloc, hipFree or other allocating
 * routine.  Its workspace is a device array of the library (64 MiB, held by each GPU the library runs on
 * until the process ends; the call takes its address on the current device) and its host staging is
 * static.  Limits: at most 16384 seeds, and the workspace of rw_solve_workspace_bytes without the
 * choice-of-m arrays (N bytes x 2 plus about 16 S m + 40 m^2 doubles) within 64 MiB; beyond them the call
 * fails with RW_EWORKSPACE.  Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (each call initializes what it reads); calls are serialized by a process-wide lock and each
 * waits for its stream before it returns, also when it fails.  Arguments, outputs and errors as for
 * rw_solve_seeds.  The call synchronizes `stream`. */
int rw_solve_seeds_noalloc(rw_graph g, const void* Q, int q_dtype, const double* lambda, int m,
                           const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C, void* U,
                           hipStream_t stream, rw_solve_info* info);

/* ======================================================================================
 * Exact random walker by conjugate gradients (Sec. II-A eq. (5), gamma = 0)
 * ====================================================================================== */
typedef struct {
  int32_t iters;        /* CG iterations (max over labels) */
  double rel_residual;  /* max over labels of ||b - L_n u|| / ||b|| */
} rw_cg_info;

int rw_cg_workspace_bytes(rw_graph g, int C, size_t* bytes);

/* Solve L_n U_n = -B^T U_s for every label by Jacobi-preconditioned CG in FP64 to a relative
 * residual <= tol (max_iter iterations at most).  U: device C x N FP64; if x0_given != 0 its
 * non-seed entries are the initial guess, else CG starts from 0.  Seed rows are one-hot on exit.
 * The call synchronizes `stream`.  Errors: RW_EINVAL, RW_EWORKSPACE, RW_ENOCONV. */
int rw_cg_solve(rw_graph g, const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C,
                double tol, int max_iter, int x0_given, double* U, void* work, size_t work_bytes,
                hipStream_t stream, rw_cg_info* info);

/* Same solver for an explicit right-hand side: L_n X_n = B_n (B: device C x N FP64, its seed rows are
 * ignored); X (device C x N FP64) is zero on the seed rows on exit, and its non-seed entries are the
 * initial guess when x0_given != 0.  Used for the adjoint system of the gradient form. */
int rw_cg_solve_rhs(rw_graph g, const int64_t* seed_node, const int32_t* seed_label, int64_t S, int C,
                    const double* B, double tol, int max_iter, int x0_given, double* X, void* work,
                    size_t work_bytes, hipStream_t stream, rw_cg_info* info);

/* ======================================================================================
 * Differentiation of the exact random walker (adjoint of Sec. II-A eq. (5), gamma = 0)
 * ====================================================================================== */

/* Replace the per-edge scales s_e (device ndir x N, FP64; entries of absent edges are ignored;
 * s_e >= 0 is the caller's responsibility) and rebuild the weights w_e = s_e exp(...). */
int rw_graph_set_scale(rw_graph g, const void* scale, hipStream_t stream);

int rw_grad_workspace_bytes(rw_graph g, size_t* bytes);

/* Given the exact solution U (device C x N FP64) and the adjoint A = L_n^{-1} G (device C x N FP64, zero
 * on seeds) of a loss gradient G = dl/dU, write (all device FP64):
 *   dw (ndir x N): dl/dw_e = -sum_k (a_i^k - a_j^k)(u_i^k - u_j^k) for each present edge e = (i, j), 0 elsewhere;
 *   ds (ndir x N): dl/ds_e = dl/dw_e exp(-beta f(J_i - J_j));
 *   dJ (N): dl/dJ through every incident edge;   dbeta (1): dl/dbeta.
 * Needs an FP64 graph.  Fixed-order reductions: the results are bitwise reproducible. */
int rw_grad_edges(rw_graph g, const double* U, const double* A, int C, double* dw, double* dJ, double* dbeta,
                  double* ds, void* work, size_t work_bytes, hipStream_t stream);

int rw_spectral_workspace_bytes(rw_graph g, int m, int C, size_t* bytes);

/* Truncated spectral approximation of the operator's pseudo-inverse applied to B (device C x N FP64):
 * X = S Q' Lambda'^{-1} Q'^T S B with Q' = columns 1..m-1 of Q (device column-major N x m FP64, column
 * 0 the null vector), S = D^{-1/2} (normalized graph) or I.  Used as the starting point of adjoint
 * solves, reusing the precomputed eigenbasis. */
int rw_spectral_apply(rw_graph g, const double* Q, const double* lambda, int m, const double* B, int C,
                      double* X, void* work, size_t work_bytes, hipStream_t stream);

/* ======================================================================================
 * Precision form: BF16 copies of the eigenbasis and matrix-core contractions with it
 * ====================================================================================== */

/* Convert a column-major rows x cols block between RW_F64 / RW_F32 / RW_BF16 (round to nearest even;
 * device buffers, src != dst).  Used to make the BF16 copy of Q that rw_solve_seeds reads with
 * q_dtype = RW_BF16: its reconstruction U = D^{-1/2} Q Y then runs on the matrix cores
 * (v_mfma_f32_16x16x16bf16, FP32 accumulation; Y split into two BF16 parts) for C <= 8.
 * dst_dtype = RW_BF16_PAIR (src RW_F64 or RW_F32) writes the pair form: dst holds
 * rows x (RW_PAIR_COLS + cols) BF16 values. */
int rw_convert_block(const void* src, int src_dtype, void* dst, int dst_dtype, int64_t rows, int cols,
                     hipStream_t stream);

int rw_project_workspace_bytes(int64_t N, int m, int C, size_t* bytes);

/* Projection onto the eigenbasis, P = Q^T X (the contraction behind eq. (16)'s Q_n^T P_n term):
 * Q device column-major N x m of q_dtype (RW_BF16: matrix cores, FP32 accumulation, X split into two
 * BF16 parts, C <= 8, m <= 256; RW_F32: FP64-accumulated VALU), X device C x N FP32, P device m x C
 * FP64 (column-major).  Fixed-order reduction of the partial sums. */
int rw_project_basis(const void* Q, int q_dtype, int64_t N, int m, const float* X, int C, double* P,
                     void* work, size_t work_bytes, hipStream_t stream);

/* ======================================================================================
 * Batching form: the online solve of Sec. II-B (gamma = 0, m fixed per image) for many images of
 * uneven sizes at once, one interaction round per enqueue, capturable into a HIP graph
 * ====================================================================================== */
typedef struct rw_batch_s* rw_batch;

typedef struct {
  rw_graph g;            /* the image's graph (all images: one graph dtype) */
  const void* Q;         /* device column-major N x m basis of q_dtype (column 0 the null vector); with the
                            graph, fixed for the batch's lifetime (rw_batch_create takes the constants
                            of its FP64 form, as rw_solve_seeds does per call) */
  int32_t q_dtype;       /* RW_F64, RW_F32 or RW_BF16 (all images: one q_dtype; not the pair form) */
  const double* lambda;  /* device FP64, m eigenvalues, lambda[0] = 0 */
  int32_t m;             /* pairs used (no choice of m in the batched form), 2 <= m <= min(N, 1024) */
  int64_t S_cap;         /* most distinct seeds this image will get in any round */
  int32_t C_cap;         /* most labels in any round, 1..8 */
  void* U;               /* device C_cap x N of the graph dtype; round output in the first C rows */
} rw_batch_image;

int rw_batch_workspace_bytes(const rw_batch_image* imgs, int n, size_t* bytes);

/* Lay out the batch inside `work` (device, rw_batch_workspace_bytes; owned by the caller, kept alive
 * until rw_batch_destroy), upload the per-image descriptors and choose the reconstruction's launch
 * shape (threads per block x nodes per thread) by timing the candidates on this batch, unless the
 * process already tuned the same batch shape (or the file named by RW_AUTOTUNE_CACHE lists it).
 * The graphs, bases and outputs must stay alive and unmoved while the batch exists.  Synchronizes
 * `stream`.  Errors: RW_EINVAL (1 <= n <= 65535, sizes, mixed dtypes), RW_EWORKSPACE, RW_EHIP. */
int rw_batch_create(const rw_batch_image* imgs, int n, void* work, size_t work_bytes, hipStream_t stream,
                    rw_batch* out);
int rw_batch_destroy(rw_batch b);

/* Launch shape in use and whether rw_batch_create timed it (tune_us: microseconds spent). */
int rw_batch_info(rw_batch b, int* threads, int* nodes_per_thread, int* tuned_now, double* tune_us);

/* Seeds of the next round (host arrays): image i has C[i] labels and the seeds
 * seed_node[seed_off[i] .. seed_off[i+1]) with labels seed_label[...], under the same rules as
 * rw_solve_seeds (validated here; nothing is changed on error).  The arrays are copied to the
 * device on `stream`, which is then synchronized: work that still reads the previous round must be
 * ordered before this call (same stream) or finished.  Errors: RW_EINVAL, RW_EHIP. */
int rw_batch_set_seeds(rw_batch b, const int* C, const int64_t* seed_off, const int64_t* seed_node,
                       const int32_t* seed_label, hipStream_t stream);

/* Enqueue one round for every image on `stream` (no host synchronization, no allocation, no
 * memset, no host-read sizes: launch shapes depend on the capacities only, so a stream capture of
 * this call replays correctly for every later round of rw_batch_set_seeds).  Per image: seed map,
 * gather of Q_s and B Q_n, the reduced system (Lambda - Q_s^T B Q_n) Y = Q_s^T op_ss U_hat_s (FP64,
 * LU with partial pivoting), and U = D^{-1/2} Q Y on non-seeds, one-hot on seeds.  Errors: RW_EINVAL
 * (no seeds set yet). */
int rw_batch_enqueue(rw_batch b, hipStream_t stream);

/* After a round has run: smallest LU pivot ratio over the images (synchronizes `stream`).
 * Errors: RW_ESINGULAR when some image's reduced system was singular (its U is then not valid). */
int rw_batch_status(rw_batch b, double* min_pivot, hipStream_t stream);

/* ======================================================================================
 * Dense FP64 building blocks used by the steps above (exposed for testing and reuse)
 * ====================================================================================== */

/* Symmetric eigendecomposition of `count` matrices A (device, n x n column-major each, stride n*n,
 * read only; only the symmetric part is used) by the parallel cyclic Jacobi method: w (device,
 * count x n, ascending) and V (device, count x n x n eigenvectors as columns, or null).  1 <= n <= 1022.
 * work: device buffer of rw_dense_syev_workspace_bytes.  Errors: RW_EINVAL, RW_EWORKSPACE. */
int rw_dense_syev_workspace_bytes(int n, int count, size_t* bytes);
int rw_dense_syev(const double* A, double* w, double* V, int n, int count, void* work, size_t work_bytes,
                  hipStream_t stream);

/* Symmetric eigendecomposition of one matrix A (device, n x n column-major, read only; only the
 * symmetric part is used) through its tridiagonal form: Householder reduction A = U T U^T (Golub & Van
 * Loan Sec. 8.3.1), eigenvalues of T by bisection on Sturm counts (Sec. 8.4.1), eigenvectors of T by
 * inverse iteration, V = U Z.  w (device, n, ascending) and V (device, n x n, eigenvectors as columns);
 * w, V and work do not overlap one another.  3 <= n <= 256 (up to 224 the reduction holds the matrix in
 * registers; above, the first n - 199 columns are reduced in global memory, the rest in LDS).
 * Inverse iteration needs separated eigenvalues: when two are closer than 1e-6 of the
 * largest Gershgorin row sum it returns RW_ENOCONV (w holds the eigenvalues; V is not reliable) and the
 * Jacobi routine above should be used.  work: device buffer of rw_dense_syev_tridiag_workspace_bytes.
 * Synchronizes `stream`.  Errors: RW_EINVAL, RW_EWORKSPACE, RW_ENOCONV. */
int rw_dense_syev_tridiag_workspace_bytes(int n, size_t* bytes);
int rw_dense_syev_tridiag(const double* A, double* w, double* V, int n, void* work, size_t work_bytes,
                          hipStream_t stream);

/* Eigenvalues and rotated right-hand sides of a batch of symmetric matrices through their tridiagonal
 * forms, the per-candidate eigenproblem of the choice of m (Sec. III-A1: one eigendecomposition per
 * candidate serves the secular equations of all labels).  Matrix b (device, column-major, leading
 * dimension ld, matrices ld*ld apart, read only) has order sizes[b] (host array, 3 <= sizes[b] <= min(ld,
 * 199)); its right-hand sides R_b (device, ld x nrhs column-major, batches ld*nrhs apart) are replaced by
 * V_b^T R_b and w_b (device, ld per matrix) receives the eigenvalues in ascending order; rows
 * sizes[b] .. ld-1 of both are set to zero.  1 <= count <= 32.  When two eigenvalues of some matrix are
 * closer than 1e-6 of its largest Gershgorin row sum the call returns RW_ENOCONV and leaves w and R
 * unchanged (the Jacobi routine serves then).  work: device buffer of
 * rw_dense_eig_rhs_batched_workspace_bytes(max size, count, nrhs).  Synchronizes `stream`.
 * Errors: RW_EINVAL, RW_EWORKSPACE, RW_ENOCONV. */
int rw_dense_eig_rhs_batched_workspace_bytes(int nmax, int count, int nrhs, size_t* bytes);
int rw_dense_eig_rhs_batched(const double* A, int ld, const int* sizes, int count, double* R, int nrhs, double* w,
                             void* work, size_t work_bytes, hipStream_t stream);

/* Solve A X = B by LU with partial pivoting (device, A n x n and B n x nrhs column-major, both
 * overwritten; X returned in B).  stat (device, 1 double) = min |pivot| / max |a_ij|, or 0 when a pivot
 * falls below 1e-14 max |a_ij| (B is then not a solution). */
int rw_dense_lu_solve(double* A, int n, double* B, int nrhs, double* stat, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* RW_H */
