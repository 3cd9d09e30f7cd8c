"""SMS-MUSSELS IRLS solver on MI355X (gfx950): HIP kernels behind a C ABI
(include/smsm.h, libsmsm.so) and a ctypes binding."""
from .smsm import (  # noqa: F401
    ABI_SYMBOLS, Geometry, Params, Plan, SmsmError, LIB_PATH, lib, make_params, status_string,
    SMSM_OK, SMSM_E_INVALID, SMSM_E_UNSUPPORTED, SMSM_E_NOMEM, SMSM_E_DEVICE, SMSM_E_NUMERIC,
    SMSM_E_NOT_CONVERGED, SMSM_E_SCRATCH, SMSM_FLAG_X_C128, SMSM_FLAG_REG_F32, SMSM_FLAG_GRAM_BF16,
)
