"""MI355X (gfx950) back-transformation of eigenvectors from tridiagonal to
band form: the hot step of the two-stage Hermitian eigensolver (Kus et al.,
"Optimizations of the Eigensolvers in the ELPA Library", Sec. 2 and 3.1).

Thin ctypes binding of the C ABI in include/elpa_hh.h.  Every step of the
computation runs in the HIP library libelpahip.so; this module only
marshals torch tensors (device memory, streams) into pointers and sizes.
There is no CPU fallback: if the library is missing, import of the binding
functions raises.
"""
from .binding import (  # noqa: F401
    AUTOTUNE_FAST, AUTOTUNE_MEDIUM, Autotune, Batch,
    BATCH_AUTO, BATCH_DIAGONAL, BATCH_ONE_LAUNCH, C64, ORDER_AUTO, ORDER_LINEAR, ORDER_XCD, PATH_AUTO, PATH_REF, PATH_SPLIT, PATH_STRIPE, PATH_WY,
    R32, R64, ElpaError, band_to_tridiag, bt2_trafo, full_to_band, cholesky_inverse,
    generalized_to_standard, generalized_back, tridiag_eigh, eigenvectors,
    generalized_eigenvectors, bt2_workspace_bytes, hh_trafo,
    hh_trafo_batched, hh_trafo_batched_ptr, chosen_plan, hh_trafo_noalloc_ptr, hh_trafo_ptr, library, library_path, num_reflectors, plan_supported,
    profile_enable, profile_last, slot_offset, strerror, version, workspace_bytes,
    workspace_bytes_batched, workspace_cached, workspace_release, tune, tune_batched, tuner_clear, tuner_get, tuner_load, tuner_save, tuner_set,
    tuner_size, NOALLOC_SCRATCH_BYTES,
)
