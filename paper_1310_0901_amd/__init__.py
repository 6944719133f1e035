"""MI355X transfer checker: Memcheck-style validation of host/device copies
(Cudagrind, arXiv 1310.0901) on gfx950.

Importing the package loads nothing native; `paper_1310_0901_amd.xfercheck`
loads the HIP library and fails loudly when it is missing.
"""
