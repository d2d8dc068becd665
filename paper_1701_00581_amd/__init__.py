"""Speckle-masking burst reconstruction on AMD MI355X (gfx950).

The computation lives in ``libnvsm.so`` (hand-written HIP kernels behind a
C ABI, declared in ``include/nvsm.h``).  This package is the thin Python
binding: ``_lib`` mirrors the C entry points one to one, and ``Session``
only allocates the device buffers (torch tensors) those calls need.
"""
from ._lib import (  # noqa: F401
    EXPORTS, LIB_PATH, NVSM_F32, NVSM_U16, Burst, NvsmError, Params, PlanInfo, default_params, lib,
    nvsm_accumulate, nvsm_autotune, nvsm_batch_plan, nvsm_bispectrum_index, nvsm_create, nvsm_destroy, nvsm_last_error,
    nvsm_plan, nvsm_prepare, nvsm_profile_enable, nvsm_profile_read, nvsm_reconstruct, nvsm_reconstruct_noalloc,
    nvsm_reconstruct_batch, nvsm_set_launch, nvsm_solve, nvsm_tune_radius, nvsm_tune_radius_plan, nvsm_stream_add, nvsm_stream_finish,
    nvsm_stream_plan, nvsm_synthesize, nvsm_w_index, nvsm_model_stf, nvsm_model_stf_plan,
    nvsm_seeing, nvsm_seeing_plan, seeing_default_params, SeeingParams, status_string, STAGES,
)
from .session import Session  # noqa: F401
