"""MI355X particle-mesh charge equilibration (QEq) for 4G-HDNNP electrostatics.

The compute path is the HIP library ``libqeq.so`` (C ABI in include/qeq.h);
``qeq`` is its ctypes binding.
"""
from . import qeq  # noqa: F401
from .qeq import Plan, QEqError  # noqa: F401
