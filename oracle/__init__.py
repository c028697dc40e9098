"""FP64 CPU oracle for the propagation of a planar source's cross-spectral density (CSD).

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, calls or links this
package. Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it. It shares no code with the HIP path; the two meet only in the seeded
input generators of ``wolf_inputs``.

Every routine follows a passage of Magalhaes & Rebordao, "PyWolf: A PyOpenCL implementation
for simulating the propagation of partially coherent light" (arXiv 2203.02734). Citations name
the section, equation or algorithm. See ``oracle.wolf_oracle`` for the readings taken where the
paper is garbled or silent.

Every function is pinned by ``tests/test_oracle_pins.py`` against closed forms, invariants and
the paper's printed numbers.
"""
from .wolf_oracle import *  # noqa: F401,F403
