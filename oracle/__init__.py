"""FP64 CPU oracle for sparse sampling and completion of VPL lighting matrices.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP path; the only
thing both sides read is the seeded input generator (``scenegen``), which
holds none of the method's arithmetic.

Every function follows the paper (Huo, Wang, Liu, Bao, "Sparse Sampling and
Completion for Light Transport in VPL-based Rendering", arXiv 2202.12567)
in its own order and notation and cites the passage it implements:

* ``philox``    -- the counter-based generator the method's random draws use
                   (Salmon et al., SC'11), pinned against numpy's Philox.
* ``shading``   -- lighting-matrix entries A(i, j) (Sec. 3) with shadow-ray
                   visibility, brute force over every sphere.
* ``cluster``   -- cluster representative and intensity (Sec. 4, I_f = I_a + I_b).
* ``lightcut``  -- the global light cut (Sec. 3 step 1, Sec. 6): conservative
                   error bound, level-by-level split test, the cap.
* ``coarsen``   -- per-slice light coarsening over the tree above the global
                   cut (Sec. 4: eps, the recursive cost, merge order) and the
                   first pass its pixel draws give (Sec. 5).
* ``sampling``  -- first uniform pass, importance g(j) = max C_j - min C_j and
                   the second pass (Sec. 5, Eq. pdf).
* ``adm``       -- non-negative completion by ADM (Appendix A), and the same
                   iteration with the non-negativity switched off.
* ``als``       -- per-row masked ALS with weighted regularisation, a
                   completion variant compared with the ADM on equal terms.
* ``render``    -- I(s) = X (Y e) (Sec. 3, step 5), the whole frame, and the
                   brute-force column sum the method approximates.
* ``mlp``       -- the learned second-pass proposal (motivated by the
                   image-space-guided sampling the conclusion names as future
                   work); forward, backward and Adam in FP64.

Parity status per function is stated in each module header.
"""
