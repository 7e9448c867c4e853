"""MI355X-native exact Gaussian-process regression (squared-exponential
kernel): covariance assembly, tiled Cholesky, triangular solves, predictive
mean and full posterior covariance, as hand-written HIP kernels for gfx950
behind the C ABI in include/gpr.h.

The kernels live in libgpr.so (built in-tree by ``build.build()``); this
package only marshals arguments. Importing it does not require a GPU; the
calls that compute do, and they fail loudly when the library is missing."""
from .gpr import (GPRError, Context, Tiled, NLML, schedule_describe, adjoint_describe,  # noqa: F401
                  persist_describe, solve_plan_describe, PRECISIONS)
from ._lib import (GPR_FP64, GPR_MIXED_FP32, GPR_MIXED_BF16, GPR_EXEC_STREAMS,  # noqa: F401
                   GPR_EXEC_PERSISTENT, GPR_EXEC_AUTO, GPR_STATE_K, GPR_STATE_L, GPR_ENOTPD,
                   GPR_EINVAL, GPR_ENODEV, GPR_ENOTSUP)
