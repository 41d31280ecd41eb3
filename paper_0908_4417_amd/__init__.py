"""MI355X-native FSPB dose-deposition coefficients (Gu et al., arXiv:0908.4417).

Thin Python binding over ``libfspb.so`` (C ABI declared in ``include/fspb.h``).
Every step of the path runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory and streams.

Low level: ``fspb_plan_create``, ``fspb_raytrace``, ``fspb_dose_coeffs``,
``fspb_plan_destroy``, ``fspb_plan_info``, ``fspb_plan_get_tables`` mirror the
C functions of the same names.

High level: ``Plan(problem, device)`` owns a torch workspace and returns CSR
tensors from ``Plan.compute()``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from ._lib import (FSPB_OK, FSPB_ERR_INVALID, FSPB_ERR_STATE, FSPB_ERR_CAPACITY, FSPB_ERR_HIP,
                   FSPB_ERR_NOMEM, FSPB_ERR_OVERFLOW, FSPB_DEPTH_TRILINEAR, FspbError, FspbGrid, FspbBeam, FspbKernel,
                   FspbPlanDesc, FspbTiming, lib, library_path, EXPORTED,
                   fspb_plan_create, fspb_raytrace, fspb_dose_coeffs, fspb_plan_destroy,
                   fspb_plan_info, fspb_plan_get_tables, fspb_plan_set_timing, fspb_plan_get_timing,
                   fspb_status_string, fspb_last_error)
from .plan import Plan, CSR, VoxelCSR, Batch, Surrogate
from ._lib import (FspbBatchConfig, fspb_batch_create, fspb_batch_nnz, fspb_batch_bind, fspb_batch_tune,
                   fspb_batch_get_config, fspb_batch_set_config, fspb_batch_run, fspb_batch_check,
                   fspb_batch_destroy, FspbTrainConfig, SURROGATE_PARAMS, fspb_surrogate_create,
                   fspb_surrogate_targets, fspb_surrogate_forward, fspb_surrogate_gradient,
                   fspb_surrogate_train, fspb_surrogate_get_params, fspb_surrogate_set_params,
                   fspb_plan_set_surrogate, fspb_surrogate_destroy, fspb_fluence_dose,
                   fspb_fluence_gradient, fspb_csr_transpose, fspb_voxel_dose, fspb_dose_coeffs_rows,
                   fspb_row_ranges, fspb_csr_transpose_noalloc, NOALLOC_SCRATCH_BYTES)

__all__ = [
    "Plan", "CSR", "VoxelCSR", "Batch", "Surrogate", "FspbError", "FspbBatchConfig", "FspbTrainConfig",
    "SURROGATE_PARAMS", "fspb_surrogate_create", "fspb_surrogate_targets", "fspb_surrogate_forward",
    "fspb_surrogate_gradient", "fspb_surrogate_train", "fspb_surrogate_get_params",
    "fspb_surrogate_set_params", "fspb_plan_set_surrogate", "fspb_surrogate_destroy",
    "fspb_fluence_dose", "fspb_fluence_gradient", "fspb_csr_transpose", "fspb_voxel_dose",
    "fspb_dose_coeffs_rows", "fspb_row_ranges", "fspb_csr_transpose_noalloc", "NOALLOC_SCRATCH_BYTES",
    "fspb_batch_create", "fspb_batch_nnz", "fspb_batch_bind", "fspb_batch_tune", "fspb_batch_get_config",
    "fspb_batch_set_config", "fspb_batch_run", "fspb_batch_check", "fspb_batch_destroy", "lib", "library_path", "EXPORTED",
    "fspb_plan_create", "fspb_raytrace", "fspb_dose_coeffs", "fspb_plan_destroy",
    "fspb_plan_info", "fspb_plan_get_tables", "fspb_plan_set_timing", "fspb_plan_get_timing",
    "fspb_status_string", "fspb_last_error", "FspbTiming",
    "FSPB_OK", "FSPB_ERR_INVALID", "FSPB_ERR_STATE", "FSPB_ERR_CAPACITY", "FSPB_ERR_HIP",
    "FSPB_ERR_NOMEM", "FSPB_ERR_OVERFLOW",
]
