"""Batched rigid-body physics step for MI355X (gfx950): HIP kernels behind a C ABI.

``rbstep`` is the ctypes binding of ``librbstep.so`` (see ``include/rbstep.h``).
"""
from .rbstep import (Batch, Contacts, Model, Multi, RbError, PARAM_FRICTION, PARAM_MASS_SCALE,  # noqa: F401
                     PARAM_GEOM_SIZE, PARAM_BODY_POS, PARAM_ACT_KP, PARAM_ACT_KD,
                     ORDER_BATCH, ORDER_HEAVY_FIRST, ORDER_INTERLEAVE, STATUS_CONOVERFLOW, STATUS_ITERCAP,
                     STATUS_NONFINITE, lib)
