"""Plain FP64 CPU oracle for the ADAGIO hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls this package; only the test suite,
the smoke check and the CPU-baseline leg of the benchmark do.  It shares no
code, tables or constants with the GPU path.

What it computes, each step following the paper (Blasiok & Tsourakakis,
"ADAGIO: Fast Data-aware Near-Isometric Linear Embeddings", arXiv 1609.05388):

* ``pca``         -- centring and the d x d covariance of the centred points
                     (Sec. 2, PCA paragraph, eq. 4) and its eigendecomposition
                     sorted by decreasing eigenvalue (top principal subspace,
                     Sec. 3 opening paragraph).
* ``jl_signs``    -- the +-1/sqrt(k) Johnson-Lindenstrauss matrix of Lemma 1 /
                     Algorithm 1, drawn from a counter-based SplitMix64.
* ``embedding``   -- Algorithm 1's map w -> (P w, S (w - P^T P w)) with the
                     floor(r/2) / ceil(r/2) split of Sec. 4.1 "Implementation".
* ``certificate`` -- eq. (3): the maximum over all unordered pairs of the
                     eq. (2) distortion, by direct differences in FP64 (C).
* ``search``      -- smallest-r search for a target distortion (Sec. 4.3,
                     Fig. 6; Table 3 of Sec. 4.4), by bisection over r.
* ``mlp``         -- FP64 forward/backward of the learned dimension predictor
                     (a method extension; not in the paper).
* ``sketch``      -- the predictor's input features (a method extension).
* ``fp8``         -- the e4m3 operand encoding of the FP8 screen (OCP FP8).
* ``rpca``        -- the randomized PCA of Sec. 4.5's Adagio-Randomized-PCA.
* ``knn``         -- exact k-nearest-neighbour queries and the majority vote
                     of Secs. 4.6 and 4.7's applications.

Readings of the paper where it is silent or garbled are listed in each
module header.
"""
