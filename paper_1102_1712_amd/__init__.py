"""MI355X-native per-projection solve of the PCA lung-motion method of
Li et al., "3D tumor localization through real-time volumetric x-ray imaging
for lung cancer radiotherapy".

The compute path is the HIP library ``libpcasolve.so`` (C ABI declared in
``include/pcasolve.h``); ``binding`` is its thin Python layer over PyTorch
device memory and streams; ``synth`` draws seeded synthetic inputs.
"""
from . import binding, synth  # noqa: F401
from .binding import (PcasError, Server, default_opts, drr_adjoint, drr_forward,  # noqa: F401
                      drr_siddon, grad_w, objective_gradient, paper_opts, pca_dvf, ray_table,
                      residual_fit, solve_projection, solve_projection_workspace,
                      tumour_position, warp_pca, warp_trilinear)

__all__ = ["binding", "synth", "PcasError", "default_opts", "paper_opts", "ray_table", "pca_dvf",
           "warp_trilinear", "warp_pca", "drr_forward", "drr_adjoint", "residual_fit", "grad_w",
           "tumour_position", "solve_projection", "solve_projection_workspace", "drr_siddon",
           "objective_gradient", "Server"]
