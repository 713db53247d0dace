"""MI355X-native hot path of full-3D SPARKLING: energy, gradient, projection, step.

The compute runs in libsparkling.so (hand-written HIP for gfx950); this package
is its ctypes binding plus the seeded input generators and workload table.
"""
from .api import (FLAG_DISCREPANCY, FLAG_LOG_KERNEL, FLAG_ROTATION_VARIANT, KERNELS, KIND_ATTRACTION, KIND_INTERPOLATION, KIND_OTHER, KIND_PROJECTION, KIND_REPULSION,
                  PRECISIONS, Params, SparklingEnergy, SparklingError, StepGraph, StepState, alpha_beta,
                  attraction_field, constraint_check, energy, grad, lipschitz_bound, load_library, project_, sparkling_energy, step_,
                  step_async_, step_async_noalloc_, noalloc_scratch_bytes, info_dict, new_duals, pair_issue_bound, probe_pair_mix, timing_enable, timing_query, timing_reset, upsample, workspace, workspace_size)

__all__ = [
    "FLAG_DISCREPANCY", "FLAG_LOG_KERNEL", "FLAG_ROTATION_VARIANT", "KERNELS", "KIND_ATTRACTION", "KIND_INTERPOLATION", "KIND_OTHER", "KIND_PROJECTION", "KIND_REPULSION",
    "PRECISIONS", "Params", "SparklingEnergy", "SparklingError", "StepGraph", "StepState", "alpha_beta",
    "attraction_field", "constraint_check", "energy", "grad", "lipschitz_bound", "load_library", "project_", "sparkling_energy", "step_",
    "step_async_", "step_async_noalloc_", "noalloc_scratch_bytes", "info_dict", "new_duals", "pair_issue_bound", "probe_pair_mix", "timing_enable", "timing_query", "timing_reset", "upsample", "workspace", "workspace_size",
]
