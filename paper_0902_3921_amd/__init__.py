"""MI355X (gfx950) implementation of the hybrid free-energy lattice Boltzmann
timestep of Tiribocchi, Stella, Gonnella and Lamura (arXiv:0902.3921).

The method runs in hand-written HIP kernels behind the C ABI of
``include/hlb.h`` (``libhlb.so``); ``paper_0902_3921_amd.hlb`` is its Python
binding.
"""
from . import hlb  # noqa: F401
from .hlb import Batch, Sim, params, check_params, workspace_size, batch_workspace_size, version  # noqa: F401
