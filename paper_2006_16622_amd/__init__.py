"""MI355X (gfx950) library for Metropolis-Hastings Monte Carlo of point
charges in a periodic cube with the multilevel local-expansion method of
Saunders, Grant & Mueller (arXiv:2006.16622).

The work runs in hand-written HIP kernels behind the C ABI of
``include/fmm_mc.h`` (``libfmm_mc.so``); this package only marshals
arguments (``binding``) and uses PyTorch for device memory and streams.
There is no CPU fallback: without the built library every call raises.
"""
from .binding import (FMM_MC_DIRECT_SETUP, FMM_MC_FREE_SPACE, FMM_MC_MIXED, FMM_MC_MULTIPOLE, FmmMcError, Chain, load_library, run_chains,  # noqa: F401
                      setup_batch, host_operator, workspace_bytes)
