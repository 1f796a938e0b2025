"""MI355X (gfx950) differentiable Gaussian-splatting hot path of 4DGCPro.

The compute runs in the HIP library ``libgs4d.so`` behind the C ABI of
``include/gs4d.h``; this package only marshals arguments to it. Importing the
package does not require a GPU; calling a render entry point does, and fails
loudly if the library has not been built.
"""
from .render import (LossWorkspace, RenderFunction, RenderSettings, Workspace, autotune, autotune_cached, color_loss,
                     deterministic, render, render_backward, render_forward, work_counters)

__all__ = ["LossWorkspace", "RenderFunction", "RenderSettings", "Workspace", "autotune", "autotune_cached", "color_loss",
           "deterministic", "render", "render_backward", "render_forward", "work_counters"]
