"""MI355X-native signature kernels by local Neumann-series propagation
(arXiv 2502.20392).  The compute path is libsigk.so (hand-written HIP for
gfx950) behind the C ABI of include/sigk.h; this package is its Python
binding (PyTorch for device memory and streams) plus autograd wrappers."""
from .api import (OrderClassPlan, RaggedPlan, backward, counters, estimate_order,  # noqa: F401
                  gram, gram_ragged, gram_static, last_autograd_counters, last_workspace, mmd2, order_bound, pair,
                  pair_backward, pair_backward_workspace_size, ragged, sigkernel_gram, workspace)
from . import _lib  # noqa: F401
