"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package only *draws inputs*: geometry, event parameters, blended
interference, trace masks and random vectors. It holds none of the
Radon-operator or inversion arithmetic, so both the FP64 oracle and the HIP
library can be fed from it without sharing any code with each other.
"""

from .configs import (  # noqa: F401
    Workload,
    workload,
    WORKLOADS,
)
from .gathers import (  # noqa: F401
    Gather,
    ricker,
    render_events,
    make_gather,
    make_cfg3_batch,
    batch_shapes,
    random_model,
    random_data,
)
from .survey import Survey, make_survey  # noqa: F401,E402
