"""Plain FP64 CPU oracle of the compact fourth-order staggered scheme.

TEST INFRASTRUCTURE ONLY: the product package never imports this module.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.  See ``c4_oracle.c`` for the passage each routine follows;
``nc_oracle.py`` holds the non-compact comparison scheme NC,
``transform_oracle.py`` the transform solve of M and ``source_oracle.py`` the
2D step with a current Jz.
"""
from .oracle import (  # noqa: F401
    CLOSURE_PAPER, CLOSURE_REFLECT, LAP_TRACKED, LAP_DISCRETE, FIELDS,
    OracleProblem, build, load, pade_line,
)
