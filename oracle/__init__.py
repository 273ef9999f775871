"""CPU oracle for the CKKS hot path of PrivFT -- TEST INFRASTRUCTURE ONLY.

Imported only by tests/, __graft_entry__.smoke() and the benchmark's CPU
baseline leg.  The product path never imports it.
"""

from . import ckks  # noqa: F401
from ._ring import build  # noqa: F401
