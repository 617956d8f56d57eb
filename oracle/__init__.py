"""CPU oracle for the adaptive progressive compressor (test infrastructure only).

A plain, slow, float64/int64 NumPy implementation of what the paper's method
computes: multilevel interpolation decomposition (per-level and per-region,
Section IV), error-bounded quantization of the coefficients, coefficient
decomposition (Section V-B, Algorithm 1), generic bitplane encoding
(Section VI-C), the retrieval interpreter with max ordering (Section V-C) and
reconstruction (Algorithm 2), plus target-driven pipeline selection
(Section VI-A).

Parity unpinned: ``select_pipeline``'s vote and the greedy order in which the
interpreter takes planes.  The paper gives no example or closed form for
either (only their inputs and guarantees are pinned: plan sizes, nesting,
and the error bound of every plan).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it; the two meet only on seeded inputs from ``fieldgen``.
"""
from .scheme import Scheme, Target  # noqa: F401
from .pipeline import refactor, plan, retrieve, select_pipeline  # noqa: F401
