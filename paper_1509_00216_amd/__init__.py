"""MI355X (gfx950) two-site H_eff x and local LCC solve for MPS-LCC (arXiv:1509.00216).

`paper_1509_00216_amd.lcc` binds the C ABI of libmpslcc.so (include/mpslcc.h).
"""
__all__ = ["lcc"]
