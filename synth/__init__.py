"""Seeded synthetic inputs shared by the oracle-side and the HIP-side tests.

This module holds workload descriptions (sizes, bit lengths, seeds) and draws
random numbers.  It contains none of the scheme's arithmetic: every random
quantity the CKKS method consumes (secret, errors, masks, encryption
randomness, slot values, plaintext integers) is drawn here and handed, as the
same arrays, to both the oracle and the HIP library.
"""

from .configs import CONFIGS, WorkloadConfig  # noqa: F401
from .inputs import *  # noqa: F401,F403
