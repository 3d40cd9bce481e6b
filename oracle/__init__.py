"""CPU FP64 reference ("oracle") for the SPH + octree hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; the GPU library never imports, links or runs it.
"""
from .oracle import *  # noqa: F401,F403
