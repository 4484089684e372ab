"""Plain FP64 CPU oracle for the grouped multi-density J/K build.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_2002_00322_amd`` and never imports it.
"""
from .reference import (  # noqa: F401
    build, boys_f0, boys_fn, eri, schwarz, eri_tensor, count, jk_literal, jk_canonical,
    jk_canonical_range, jk_entries, nine_densities, energy_two_body, energy_one_body, energy_gradient,
    num_threads, primitive_overlap, contraction, eri_contracted, jk_contracted,
)
