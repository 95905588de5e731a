"""MI355X (gfx950) implementation of hypothesis-tested progressive kernel estimation (arXiv 2504.04411).

``hk`` is the ctypes binding of libhk.so (include/hk.h); ``estimator`` a torch-side buffer manager.
"""
