"""MI355X-native NEMD channel micro-solver with GP and MLP-ensemble surrogates
for the hybrid continuum-atomistic scheme of Stephenson, Kermode & Lockerby
(arXiv:1603.04628).

All computation happens in ``libhmd.so`` (hand-written HIP for gfx950, C ABI
in ``include/hmd.h``); ``binding`` only marshals arguments.  Importing the
package fails if the library is not built.
"""
from . import binding  # noqa: F401  (raises ImportError when libhmd.so is missing)
from .binding import (Batch, Context, HmdError, Params, System, md_autotune,  # noqa: F401
                      md_flux, md_flux_batch, md_flux_batch_dev)
from .binding import GP, Ensemble, ens_cfg, gp_hyper  # noqa: F401,E402
from .hybrid_binding import Hybrid, hybrid_cfg  # noqa: F401,E402
