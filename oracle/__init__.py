"""FP64 CPU oracle of the LBRMT time step -- TEST INFRASTRUCTURE ONLY.

Importable only by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py``; the GPU library never links, imports or calls it.
"""
from .oracle import Oracle, d2q9, feq_sfc, guo, heaviside, layers_mask, solid_stress  # noqa: F401
