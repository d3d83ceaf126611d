"""MI355X (gfx950) HIP implementation of the HMC volatility update of the
realized stochastic volatility model (Takaishi, arXiv:1603.08114).

The compute path is the HIP library ``librsvhmc.so`` (sources in ``csrc/``,
C ABI in ``include/rsv_hmc.h``); ``api`` is its Python binding.
"""
from ._lib import (RSV_F32_MIXED, RSV_F64, RSV_TERM_RETURN, RSV_TERM_RV,  # noqa: F401
                   RSV_TERMS_RSV, LIB_PATH, EXPORTS)

__all__ = ["RSV_F64", "RSV_F32_MIXED", "RSV_TERM_RETURN", "RSV_TERM_RV", "RSV_TERMS_RSV",
           "LIB_PATH", "EXPORTS"]
