"""FP64 CPU oracle of REFINE's scoring and pruning -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_2606_09074_amd``) and never imports it.
"""
from .oracle import (Params, activate_one, build, compact, lam, load, n_prune, nonfinite, num_threads,
                     pair, score, select, stats)

__all__ = ["Params", "activate_one", "build", "compact", "lam", "load", "n_prune", "nonfinite",
           "num_threads", "pair", "score", "select", "stats"]
