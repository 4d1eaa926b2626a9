"""CPU oracle for packed approximate convolution -- TEST INFRASTRUCTURE ONLY.

Imported only by tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py.
Shares no code with the HIP library and imports nothing from it.
"""
from .core import *  # noqa: F401,F403
from .core import _packed_core  # noqa: F401
from . import marginal  # noqa: F401
