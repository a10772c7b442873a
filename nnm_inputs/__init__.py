"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This package holds no arithmetic of the rendering method itself (no sphere
tracing, no network evaluation, no normals).  It only produces inputs:

* SIREN weights drawn with the SIREN initialisation scheme (cited in the
  paper's Related Work as the initialisation its networks use), made
  Lipschitz-safe by scaling the output layer;
* pinhole-camera rays;
* the torus training data for the fitting workload;
* the scene descriptions of the five standard workloads;
* regular grids of sample points.

All randomness comes from numpy's PCG64 (`numpy.random.default_rng`) and all
derived values are computed in float64 before being rounded once to float32.
"""

from .siren_init import (  # noqa: F401
    SirenNet,
    siren_init,
    lipschitz_product_bound,
    param_count,
    flatten_params,
    unflatten_params,
)
from .camera import pinhole_rays  # noqa: F401
from .torus import torus_sdf, torus_surface_samples, torus_uniform_samples, torus_batch  # noqa: F401
from .scenes import SceneLevel, Scene, make_scene, WORKLOADS, TABLE3_ROWS  # noqa: F401
from .netfile import write_net_file, read_net_file  # noqa: F401
from .grid import grid_axis, grid_nodes  # noqa: F401
