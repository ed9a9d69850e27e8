"""CPU FP64 oracle for the polarizability build and the screened interaction
that follows it -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the library never does.
"""
from . import chi  # noqa: F401
from . import w  # noqa: F401
from . import pade  # noqa: F401
