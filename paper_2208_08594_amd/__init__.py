"""MI355X-native multi-stage (CPR-type) preconditioned FGMRES for block-sparse
reservoir Jacobians (Zhao, Zhang, Feng, Shu: "An Improved Multi-Stage
Preconditioner on GPUs for Compositional Reservoir Simulation", 2022).

Submodules:
  synth  -- seeded synthetic Jacobian generators (inputs only; no solver arithmetic)
  msp    -- ctypes binding of the C-ABI library libmsp.so (HIP kernels for gfx950)
  serve  -- continuous-batching request loop over the C-ABI

Importing the package loads nothing; ``msp`` loads libmsp.so on first use and
raises if it is missing.
"""
__all__ = ["synth", "msp", "serve"]
