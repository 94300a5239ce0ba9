// Bank of eigenbases precomputed for several beta (Sec. III-B, last paragraph): eigenvectors for several beta
// are precomputed and the Rayleigh quotients of eq. (26) "interpolate" between them.  For the graph's current
// operator every bank basis gets the diagonal update of eq. (27) (its null vector replaced by the current one,
// the other columns re-orthonormalized in order, lambda_hat_i = q_i^T op q_i), and the basis whose quotients
// sum lowest is returned with its lambda_hat: among orthonormal bases of m columns the eigenbasis of the m
// smallest eigenvalues has the smallest sum (Ky Fan), so the sum ranks the bases by how well they span the
// current low spectrum.
#include <cmath>
#include <vector>

#include "rw_internal.h"

using namespace rw;

extern "C" {

int rw_bank_workspace_bytes(rw_graph h, int m, const rw_eig_opts* opts, size_t* bytes) {
  return rw_update_workspace_bytes(h, m, opts, bytes);
}

int rw_bank_select(rw_graph h, const void* const* Q_bank, int nbank, const rw_eig_opts* opts, int m, void* Q_out,
                   double* lambda_out, void* work, size_t work_bytes, hipStream_t stream, int* chosen,
                   double* traces) {
  RW_NOT_CAPTURING(stream);
  RW_CHECK(h != nullptr && Q_bank != nullptr && opts != nullptr && Q_out != nullptr && lambda_out != nullptr &&
               chosen != nullptr,
           RW_EINVAL, "null argument");
  RW_CHECK(nbank >= 1, RW_EINVAL, "the bank is empty");
  for (int b = 0; b < nbank; ++b) {
    RW_CHECK(Q_bank[b] != nullptr, RW_EINVAL, "bank basis %d is null", b);
    RW_CHECK(Q_bank[b] != Q_out, RW_EINVAL, "Q_out must not be a bank basis");
  }
  const Graph* g = &h->g;
  const size_t qbytes = (size_t)g->N * m * dtype_size(opts->q_dtype);
  std::vector<double> lam((size_t)std::max(m, 1));
  int best = -1;
  double best_sum = INFINITY;
  // the diagonal update of basis b into Q_out, lambda_out; its quotient sum
  auto evaluate = [&](int b, double* sum) -> int {
    RW_HIP(hipMemcpyAsync(Q_out, Q_bank[b], qbytes, hipMemcpyDeviceToDevice, stream));
    RW_TRY(rw_update_eig(h, nullptr, 0, RW_UPDATE_DIAG_RQ, opts, Q_out, lambda_out, m, work, work_bytes, stream,
                         nullptr));
    RW_HIP(hipMemcpyAsync(lam.data(), lambda_out, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, stream));
    RW_HIP(hipStreamSynchronize(stream));
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += lam[i];
    *sum = s;
    return RW_OK;
  };
  for (int b = 0; b < nbank; ++b) {
    double s = 0.0;
    RW_TRY(evaluate(b, &s));
    if (traces) traces[b] = s;
    if (s < best_sum) {
      best_sum = s;
      best = b;
    }
  }
  RW_CHECK(best >= 0, RW_EINVAL, "no bank basis has a finite quotient sum");
  if (best != nbank - 1) {   // Q_out holds the last basis evaluated: redo the chosen one (same arithmetic)
    double s = 0.0;
    RW_TRY(evaluate(best, &s));
  }
  *chosen = best;
  return RW_OK;
}

}  // extern "C"
