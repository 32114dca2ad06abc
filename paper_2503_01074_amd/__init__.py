"""OceanSim sensor image formation on MI355X (gfx950).

Imaging-sonar image formation from ray-cast returns and the underwater colour
image-formation model of arXiv 2503.01074, as hand-written HIP kernels behind
the C ABI in include/oceansim.h (liboceansim.so, built in-tree).
"""
# torch first: the library then binds to the HIP runtime torch loaded (both
# name it libamdhip64.so.7; the first one loaded serves the process)
import torch  # noqa: F401,E402
from . import _lib  # noqa: F401  (fails loudly when the library is not built)
from ._lib import (OceansimError, SPECKLE_GAMMA, SPECKLE_OFF, SPECKLE_PAPER,  # noqa: F401
                   SONAR_GRAD_COLUMNS, SONAR_GRAD_WIDTH, WATER_GRAD_WIDTH)
from .api import (DeviceHits, Plan, Scene, SonarGeometry, SonarRender, UwForm, raycast, render_sonar,  # noqa: F401
                  scene_measure,
                  barometer, cam_condition, cam_condition_backward, cam_encode, dvl,
                  render_sonar_backward, sonar_params, sonar_params_from_spec, uw_form,
                  uw_form_backward, water_params)
