"""Synthetic robot descriptions and seeded inputs shared by the oracle and the HIP path.

Nothing in this package performs any step of the physics method: it only builds
model descriptions (geometry, masses, solid-shape inertias) and draws seeded
random inputs.  Both the FP64 oracle (``oracle/``) and the HIP library consume
what it produces, each through its own marshalling code.
"""
