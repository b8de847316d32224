"""Seeded synthetic instances of the Hessian equation H y = r.

This package only draws random inputs; it contains none of the method's
arithmetic.  Both the CPU oracle and the GPU library read the same FP64 bits
from it, so a parity test always compares the two on identical data.
"""

from .generator import (  # noqa: F401
    Instance,
    make_instance,
    make_path,
    draw_batch_shape,
    draw_serving_shape,
    batch_instances,
    serving_requests,
    CONFIG_C1,
    CONFIG_C2,
    CONFIG_C4,
)
