"""FP64 CPU oracle of the TOI imaging path and the FITrig stage.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the benchmark's ``cpu_baseline`` leg, never by the product path.  It shares
no code with the HIP library; only the seeded input generator
(``synth_inputs``) serves both.
"""
from . import toi, fitrig, gridded, adjoint  # noqa: F401
