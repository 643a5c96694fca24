"""FP64 CPU oracle of the MHM local problems and the skeleton system.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the library.  It shares no
code with the HIP path.
"""
from .local import local_problem, solve_batch, solve_element  # noqa: F401
