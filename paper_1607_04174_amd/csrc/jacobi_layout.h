// Position-based storage of a symmetric matrix for the round-robin Jacobi ordering.
//
// In the round-robin ("tournament") ordering of the cyclic Jacobi method (Golub & Van Loan,
// Sec. 8.5) round r pairs position k with position n2-1-k (k < n2/2), and between rounds every
// index except the one at position 0 moves down one position (position 1 wraps to n2-1).  Storing
// the matrix by position rather than by index keeps each pair's 2 x 2 blocks at fixed addresses:
// the off-diagonal block of pairs k1 < k2 is one entry in each of four arrays (slot (s1, s2), slot
// 0 = the low position k, slot 1 = the high position n2-1-k), and the diagonal block of pair k is
// three entries (aa, ab, bb).  After a round's rotations each entry is written to the position its
// indices occupy in the next round.
#pragma once
#include <hip/hip_runtime.h>

namespace rw {

struct JacLayout {
  int n2, np, nto;   // padded order (even), pairs, off-diagonal blocks
  __host__ __device__ explicit JacLayout(int n)
      : n2(n + (n & 1)), np((n + (n & 1)) / 2), nto(((n + (n & 1)) / 2) * ((n + (n & 1)) / 2 - 1) / 2) {}
  __host__ __device__ int pair(int x) const { return x < np ? x : n2 - 1 - x; }
  __host__ __device__ int slot(int x) const { return x < np ? 0 : 1; }
  __host__ __device__ int pos(int k, int s) const { return s ? n2 - 1 - k : k; }
  // position that the index now at position x occupies in the next round
  __host__ __device__ int next(int x) const { return x == 0 ? 0 : (x == 1 ? n2 - 1 : x - 1); }
  // off-diagonal block number of pairs k1 < k2
  __host__ __device__ int block(int k1, int k2) const { return ((k2 * (k2 - 1)) >> 1) + k1; }
  // flat index (in doubles) of the symmetric entry at positions (x, y)
  __host__ __device__ int at(int x, int y) const {
    int k1 = pair(x), k2 = pair(y), s1 = slot(x), s2 = slot(y);
    if (k1 == k2) return 4 * nto + (s1 == s2 ? 2 * s1 : 1) * np + k1;
    if (k1 > k2) {
      int t = k1; k1 = k2; k2 = t;
      t = s1; s1 = s2; s2 = t;
    }
    return (2 * s1 + s2) * nto + block(k1, k2);
  }
  __host__ __device__ int words() const { return 4 * nto + 3 * np; }
  // the L-th off-diagonal block (0 <= L < nto) in a folded order: column np-1-h (np-1-h blocks) and
  // column h (h blocks) share a run of np-1 consecutive numbers, so consecutive numbers mostly share k2
  // and have consecutive k1
  __host__ __device__ void unfold(int L, int& k1, int& k2) const {
    const int w = np - 1;
    const int fc = L / w, r = L - fc * w;
    if (fc < np / 2) {
      const int ac = w - fc;
      if (r < ac) { k1 = r; k2 = ac; }
      else { k1 = r - ac; k2 = fc; }
    } else {   // odd np: the middle column
      k1 = r;
      k2 = fc;
    }
  }
};

}  // namespace rw
