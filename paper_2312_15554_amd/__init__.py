"""MI355X (gfx950) unit-cell solvers for periodic porous media: Stokes flow by
ADMM and advection-diffusion by the Lippmann-Schwinger iteration, on the
extended domain with spectral (FFT) solves.  The compute runs in the HIP
library libacm.so; this package only marshals arguments to its C ABI."""

__all__ = ["abi", "api", "inputs"]
