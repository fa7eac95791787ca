"""MI355X (gfx950) solve path of matching-based AMG preconditioned CG for IgA
stiffness systems (D'Ambra, Durastante, Filippone, arXiv 2511.21268).

The product is libamgiga.so (C ABI in include/amg.h): host hierarchy set-up by
compatible weighted matching, and a solve phase made of hand-written HIP
kernels.  This package is its thin binding; `workloads` holds the seeded
synthetic inputs.
"""
from .amg import (AmgError, Context, iga_cube, iga_diffusion, iga_poisson, lib, match, paper_default,  # noqa: F401
                  params_default,
                  sell_spmv_host)

__all__ = ["AmgError", "Context", "iga_cube", "iga_diffusion", "iga_poisson", "lib", "match", "paper_default",
           "params_default", "sell_spmv_host"]
