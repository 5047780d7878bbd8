"""MI355X-native ASRAL solver for Load Balanced Demand Distribution under
overload penalties (arXiv 2304.06543).

The solver is the HIP library ``liblbdd.so`` (C ABI in ``include/lbdd.h``);
``paper_2304_06543_amd.lbdd`` is its Python binding.
"""
from .lbdd import Instance, LbddError, best_transfers, load, solve  # noqa: F401
