"""CPU complex128 oracle of the QPINN circuit hot path.

Test infrastructure only: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; never by the product path.
"""
from . import qpinn_oracle  # noqa: F401
