"""Reference oracle for the OPH / GOPH / HOPH hot path.

TEST INFRASTRUCTURE ONLY: only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of bench.py may import, call, link or run anything under
``oracle/``.  The GPU library never does, and this package imports nothing
from the library.

* ``oracle.tiny``  -- pure Python, exact fractions, the paper's definitions
  step by step; small inputs only.
* ``oracle.scale`` -- ctypes front end of ``oph_oracle.c`` (plain C, OpenMP),
  the same conventions at collection scale.
"""
