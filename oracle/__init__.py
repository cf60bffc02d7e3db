"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import this package.  It is the plain reference the HIP path is checked against and
shares no code with it.  ``Oracle`` wraps the C++ library ``librbo.so`` (built by
``oracle.build.build()``) through ctypes: argument marshalling only.

Functions without an independent pin: none beyond what the tests list; the whole
oracle's equivalence with MuJoCo itself is "parity unpinned" (MuJoCo is not available).
"""
from .pyoracle import Oracle, build_if_missing  # noqa: F401
