"""CPU FP64 oracle of the UL-PPM Newmark step -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import this package.  The GPU library never loads it.
"""
from .oracle import *  # noqa: F401,F403
