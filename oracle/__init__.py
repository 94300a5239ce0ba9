"""CPU oracle for precomputed-eigenvector random-walker segmentation (Andrews & Hamarneh,
"Adaptable Precomputation for Random Walker Image Segmentation and Registration").

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import anything from this package.  The GPU library never calls it, and it
shares no code with the GPU library (only the seeded input generators in `rwsynth` serve both).

Everything here is plain, slow FP64 numpy/scipy, written to be checked against the paper by eye:
  graph.py      image graph, weights, Laplacian L = D - W, normalized Laplacian (Sec. II-A eq. (2);
                Sec. II-C)
  exact_rw.py   basic random walker: the linear system of Sec. II-A eq. (5), by CG and direct solve
  eigen.py      the m smallest eigenpairs (Sec. II-B eq. (6)) by dense eigendecomposition, closed
                forms for beta = 0, and residual certification
  fast_rw.py    the precomputed ("fast") random walker, Sec. II-B eqs. (7)-(17), with the
                gamma = 0 null-vector treatment of the paragraph after eq. (17)
  choose_m.py   online choice of m from the seeds, Sec. III-A1 eq. (24)
  update.py     Laplacian update: Ncut / Rayleigh-quotient eigenvalue update of Sec. III-B
                eqs. (26)-(28), and Rayleigh-Ritz on the same span
  adjoint.py    exact adjoint of the basic random walker (gradients w.r.t. weights, intensities, beta)

Readings of points where the paper is silent or ambiguous are stated in each function's docstring.
"""
