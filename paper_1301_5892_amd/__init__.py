"""MI355X (gfx950) implementation of the semi-Lagrangian 1D x 1D
Vlasov-Poisson split step of "Vlasov on GPU (VOG project)".

The method runs in libvog.so (HIP kernels behind the C ABI of
include/vog.h); `vog` is its ctypes binding and `serving` the continuous-
batching request loop built on it.
"""
from .vog import (Sim, VogError, build_info, load, make_config, step_batch,  # noqa: F401
                  workspace_bytes)
