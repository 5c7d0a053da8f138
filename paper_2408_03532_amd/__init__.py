"""MI355X-native batched 2-D partial Fourier transform and PIE sweep.

The computation runs in the HIP library libpftpie.so (C ABI in
include/pftpie.h); this package only marshals torch tensors into it.
"""

from ._lib import PftpieError, lib  # noqa: F401
from .pft import (Group, Plan, PolyPlan, autotune, get_plan, grouped_workspace_bytes, pft2d,  # noqa: F401
                  pft2d_adj, pft2d_adjoint, pft2d_forward, pft2d_grouped)
from .pie import PieParams, Scan, crop_amplitudes, hybrid_pie, pie_sweep, rel_change  # noqa: F401
from .loss import AmplitudeLoss, amp_loss, amp_loss_grad, amplitude_loss  # noqa: F401
