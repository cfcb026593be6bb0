"""Plain, slow FP64 CPU oracle for the planar photoacoustic operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links anything under ``oracle/``; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark do.
The oracle shares no code with the GPU path: it imports numpy/scipy only and
takes every input (objects, noise, start vectors) as an argument.

What it computes follows the paper (arXiv 2603.28150):

* the homogeneous, lossless wave equation with p(r,0)=p0 and zero initial
  velocity (Sec. 2, eq. 1-2), solved exactly on a grid that is periodic in
  x, y and z (the semi-discrete spectral solution p^(k,t) = cos(c|k|t) p0^(k));
* its restriction to the sensor plane z = 0, which is the depth-dependent,
  transverse shift-invariant model of Sec. 2.1 (eq. 6) and its Riemann-sum
  discretisation (Sec. 2.2, eq. 7-8), with all constants absorbed in the
  kernels;
* the adjoint for the Euclidean inner products (eq. 9-11);
* the objective, gradient and FISTA iteration of Sec. 2.3 (eq. 12-15).

Modules:
  geometry   grids, wavenumbers and the default z-period of the simulation
  hlib       kernel library H^[k, l, n] by direct DFT sums; real-space kernels
  operators  A and A^T three ways: direct circular convolution sums, dense
             DFT matrices, and numpy.fft
  wave3d     an independent k-space time stepper of the 3D wave equation
  solvers    power iteration, the exact operator norm, FISTA / projected
             gradient, dense matrices for brute-force checks
  quant      16-bit storage of H^ with per-depth power-of-two scales
"""
