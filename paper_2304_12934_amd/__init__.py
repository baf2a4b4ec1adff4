"""MI355X-native NUFFT Radon projector, adjoint, qGGMRF prior and MBIR step.

The computation lives in ``libnufftradon.so`` (hand-written HIP for gfx950,
C ABI in ``include/nufftradon.h``); this package is its Python binding.
"""

from .radon import (  # noqa: F401
    MBIR,
    DataFidelityFn,
    Graph,
    HostMBIR,
    Plan,
    Prior,
    QGGMRFFn,
    RadonFn,
    SliceGeometry,
    kb_eval,
    power_lipschitz,
    qggmrf_grad,
    stream_stack,
)

__all__ = ["Plan", "Graph", "SliceGeometry", "Prior", "RadonFn", "DataFidelityFn", "QGGMRFFn", "MBIR", "HostMBIR",
           "qggmrf_grad", "power_lipschitz", "kb_eval", "stream_stack"]
