"""Plain, slow FP64 CPU oracle for H-matrix LU (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It imports nothing from the device path and the device path never
imports it.
"""
from .hmatrix import *  # noqa: F401,F403
