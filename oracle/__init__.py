"""FP64 CPU oracle of TPO (arXiv 2405.11922).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  The native library and
its Python binding never call it, and it shares no code with them: it is a
plain, slow, obviously-correct restatement of the paper in numpy/scipy,
float64 throughout.

Parity status of each function is stated in its docstring ("pinned by ..." or
"parity unpinned").
"""
from .tpo_oracle import *  # noqa: F401,F403
from .tpo_oracle import __all__  # noqa: F401
