"""CPU oracle for the selective Fock-amplitude path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything here.  The GPU library never calls it,
and it shares no code with the GPU library: it takes the Bargmann triple as
plain arrays and computes everything in float64 / complex128 with NumPy.
"""
from .fock_oracle import *  # noqa: F401,F403
