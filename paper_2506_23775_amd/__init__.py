"""MI355X-native matrix-free circuit contraction (arXiv 2506.23775).

The hot path -- cost f(G) = -Re Tr[U^dagger C(G)], Riemannian gradient,
Hessian-vector products and Hessian blocks summed over all basis states -- runs
in the HIP kernels of ``librq.so`` behind the C ABI of ``include/rq.h``;
``paper_2506_23775_amd.rq`` is its ctypes binding.
"""

__all__ = ["rq"]
