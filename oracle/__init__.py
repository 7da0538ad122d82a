"""CPU FP64 oracle for quantum PageRank (Tang et al., arXiv:2003.04930).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, calls or links it, and it
shares no code with that path.

Everything here is plain NumPy/SciPy in float64 / complex128, written from the
paper's definitions, slow and obvious on purpose.  Where the paper is garbled
the reading taken is stated in the docstring of the function that applies it.
"""
from .qpr_ref import *  # noqa: F401,F403
from .qpr_ref import __all__ as _qpr_all
from .mpnn_ref import *  # noqa: F401,F403
from .mpnn_ref import __all__ as _mpnn_all

__all__ = list(_qpr_all) + list(_mpnn_all)
