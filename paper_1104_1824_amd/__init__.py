"""MI355X (gfx950) simulator of spiking neural P systems without delays.

Breadth-first expansion of the computation tree, C' = C + S.M over every valid
spiking vector S of every frontier configuration (Cabarle, Adorna,
Martinez-del-Amor, arXiv:1104.1824), in hand-written HIP kernels behind the C
ABI of include/snp.h.  ``snp`` is the ctypes binding; ``build`` compiles the
library.
"""
from . import snp  # noqa: F401
from .snp import (  # noqa: F401
    SnpError,
    snp_expand,
    snp_free,
    snp_load,
    snp_reset,
    snp_row_bytes,
    snp_run,
    snp_run_batch,
)
