"""FP64 CPU oracle for sparse MTTKRP and CP-ALS.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``.  The library itself never imports,
links or runs anything from here, and nothing here imports the library.

* ``mttkrp`` / ``mttkrp_rows``: the definition of Eq. (1) (Sec. II-A) as a
  plain COO loop in C, FP64 accumulation (``coo_mttkrp.c``).
* ``cp_als`` and its steps: textbook CP-ALS (the survey the paper cites for
  tensor background, Kolda & Bader) in FP64 numpy (``als.py``).
* ``bf16_round``: round-to-nearest-even of FP32 to bfloat16 (``bf16.py``).
"""

from .ref import mttkrp, mttkrp_rows, lib_path  # noqa: F401
from .als import (  # noqa: F401
    cp_als, gram, hadamard_of_grams, solve_mode, normalize_columns, fit_from_parts, coalesce, AlsState,
    als_init, als_iteration,
)
from .bf16 import bf16_round  # noqa: F401
