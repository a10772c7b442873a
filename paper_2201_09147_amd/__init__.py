"""Python binding of libnnm: sphere tracing of nested SIREN SDFs on MI355X.

Argument marshalling only: every step of the path runs in the HIP kernels of
``libnnm.so`` (built by ``paper_2201_09147_amd.build``).  Importing works without
the library; the first call into it raises ``NnmError`` if it is not built.
Device arrays are torch tensors on the stack's device; streams are torch
streams (default: the current stream).

Entry points (same names as the C ABI in include/nnm.h):
  load_siren_stack, free_siren_stack, trace_rays, trace_rays_noalloc, analytic_normal,
  nnm_net_eval, nnm_sup_abs_diff, nnm_sup_abs_err, nnm_nesting_thresholds,
  neural_normal_map, nnm_grid_values,
  nnm_mesh_extract, nnm_validate_stack, nnm_read_net_file, nnm_sync
plus ``render`` (allocates outputs and calls trace_rays), ``extract_mesh`` and
``mesh_neural_normal_map`` (coarse mesh + fine normals), the fitting entry
points (``Fit`` over fit_create / fit_step, siren_forward_tangent,
siren_backward) and ``paper_2201_09147_amd.autograd.SirenFn``.
"""

from ._binding import (  # noqa: F401
    NnmError,
    LevelSpec,
    Stack,
    TraceParams,
    Profiler,
    PRECISIONS,
    ST_HIT,
    ST_FAR,
    ST_BUDGET,
    ST_NEG_STEP,
    ST_NONFINITE,
    library_path,
    load_library,
    load_siren_stack,
    free_siren_stack,
    trace_rays,
    trace_rays_noalloc,
    NOALLOC_MAX_RAYS,
    analytic_normal,
    nnm_net_eval,
    nnm_sup_abs_diff,
    nnm_sup_abs_err,
    nnm_nesting_thresholds,
    nesting_thresholds,
    capacity_thresholds,
    KERNELS,
    neural_normal_map,
    nnm_grid_values,
    nnm_mesh_extract,
    extract_mesh,
    mesh_neural_normal_map,
    nnm_validate_stack,
    nnm_level_lipschitz_bound,
    nnm_read_net_file,
    nnm_write_net_file,
    nnm_sync,
    render,
    levels_from_scene,
    Fit,
    siren_workspace_bytes,
    siren_forward_tangent,
    siren_backward,
)
