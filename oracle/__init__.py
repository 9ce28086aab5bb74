"""FP64 CPU oracle for the curvilinear lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the HIP library.
"""
from .oracle import OracleGrid, lattice, feq, build, lib_path, max_threads  # noqa: F401
from . import exact  # noqa: F401
from . import oracle3d  # noqa: F401
