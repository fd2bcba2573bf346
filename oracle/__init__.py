"""CPU FP64 oracle for the contour-FFT (C-FFT) tabulation of MBF reaction terms.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: it exists so that tests, the smoke check and the CPU
baseline leg of the benchmark can compare the GPU library against a plain,
slow, obviously correct implementation written from the paper
(Jha & Craeye, "Contour-FFT based Spectral Domain MBF Analysis of Large
Printed Antenna Arrays").

It shares no code with the HIP path: the Green's function is assembled from
transmission-line admittances (not the closed-form denominators the kernels
use), the spectra are summed basis by basis, and the table is a direct sum per
output displacement (no FFT, no sign modulation trick).

Modules
  cfft_oracle  grid, contour, Green's function, spectra, integrand, direct sum,
               bilinear lookup, loss and its gradient
  ocont        continuum reaction integral by polar quadrature along a
               deformed radial contour (accuracy reference, pins only)

Parity status of every function is stated in its docstring ("pinned by ...").
"""
