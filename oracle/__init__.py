"""FP64 CPU oracle for the RaNN overlapping-Schwarz least-squares method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and this
package never imports the product.  The two share nothing but the seeded input
generator, which holds none of the method's arithmetic.

What it computes (Shang, Heinlein, Mishra, Wang, "Overlapping Schwarz
preconditioners for randomized neural networks with domain decomposition"):

* geometry      -- subdomain supports and window-function partition of unity
                   (Sec. 2 local/global spaces; Sec. 5 Ex. 1 window formula)
* features      -- single-hidden-layer tanh RaNN features on normalised input
                   and their derivatives (eq. (rann), Sec. 5 normalisation)
* assemble      -- collocation rows A[L w_j phi] and boundary rows, the system
                   H W = F (eqs. (sum), (system)), with the PCA basis
                   (Sec. 4, eqs. (pca), (pca_net), (system_new))
* pca           -- SVD of the value matrix Psi_j and truncation (Sec. 4)
* lsq           -- the exact least-squares solution by Householder QR (the
                   paper's direct comparison solver, Sec. 5) and its adjoint
* schwarz       -- AS / RAS / SAS preconditioners (Sec. 3)
* krylov        -- CG on the normal equations and left-preconditioned GMRES
                   (Sec. 3, Sec. 5 stopping rule)
* blocksparse   -- the same operators on per-subdomain blocks for sizes where a
                   dense H does not fit

Readings of passages where the paper is silent or garbled are listed in the
design notes; each function states the one it uses.
"""
