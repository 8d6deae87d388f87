"""FP64 CPU oracle for the randomized SVD / PCA hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (``paper_1608_02148_amd``) never imports it and shares no code,
constants or helpers with it.

The oracle follows Erichson, Voronin, Brunton & Kutz, "Randomized Matrix
Decompositions Using R" (arXiv:1608.02148):

* ``philox``  -- the counter-based generator used for the Gaussian test matrix
  (Sec. 2.3 asks for i.i.d. N(0,1) entries; the generator itself is Salmon et
  al., SC'11, and Box-Muller, 1958).
* ``rsvd``    -- Alg. rqb (randomized QB), Alg. subspace_iter (subspace
  iterations), Alg. RSVDalgorithm (randomized SVD), Alg. RPCAalgorithm
  (randomized PCA), plus the diagnostics of Sec. 3.4 (Eckart-Young optimum and
  the expected-error bound, Eq. rsvd_expected_error).
* ``mlp``     -- the small fully connected network that predicts (q, p) from a
  q=0 sketch spectrum (not in the paper; written from the standard definitions
  of affine layers, ReLU, softmax cross-entropy and Adam).

Everything is plain numpy in float64.  Library primitives used as steps:
``numpy.linalg.qr`` (the paper's ``qr``), ``numpy.linalg.svd`` (the paper's
``svd``), matrix products.  No blocking, fusion or reordering beyond what the
paper's algorithms state.
"""
