"""FP64 CPU oracle for LMMSE-CG equalisation of Zak-OTFS frames.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and the
cpu_baseline leg of the benchmark may import or call anything in this package.  The HIP
library never links, imports or falls back to it, and it shares no code, table or helper
with the HIP path.
"""
from .otfs_oracle import *  # noqa: F401,F403
from .otfs_oracle import __all__  # noqa: F401
