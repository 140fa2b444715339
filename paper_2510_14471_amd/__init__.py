"""PCG-Aug GLS estimation of SUR models on MI355X (gfx950).

The compute path is the HIP library ``libglm_hip.so`` (C ABI in
include/glm.h); this package only marshals arguments to it.  Importing the
package fails if the library has not been built.
"""
from ._lib import (  # noqa: F401
    GLM_FP64, GLM_MIXED, GLM_REDUCED, GLMError, Shape, glm_copy_factors, glm_factor_destroy, glm_get_stats,
    glm_gls_backward, glm_gls_solve, glm_profile_enable, glm_profile_read,
    glm_qr_factor, glm_stream_mix, glm_strerror, glm_validate_shape, glm_workspace_bytes,
)
from .solver import (  # noqa: F401
    BatchLayout, MVRSolver, SURSolver, gls, pack_instances, pack_mvr, unpack,
)
