"""FP64 CPU oracle for NURSD / SRSD -- test infrastructure only.

Imported only by tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
leg.  The GPU product path never imports it and shares no code with it.
"""
from . import nursd_ref  # noqa: F401
