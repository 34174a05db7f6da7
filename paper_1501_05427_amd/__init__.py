"""MI355X (gfx950) implementation of the hot path of SGLD with the ULISSE solver for
Gaussian-process covariance parameters (Filippone & Engler, ICML 2015).

The computation lives in the HIP library libulisse_gp.so (sources in csrc/, C ABI in
include/ulisse_gp.h); ``binding`` exposes it to Python under the same names.
"""
from . import binding  # noqa: F401
from .binding import (  # noqa: F401
    GP_BF16_SPLIT_KV, GP_BF16_SPLIT_V, GP_FP32, Handle, colmajor, gp_create, gp_destroy,
    gp_dkmv, gp_draw_probes, gp_kmv, gp_last_error, gp_philox, gp_stoch_grad, make_params,
    sgld_step, ulisse_solve,
)
