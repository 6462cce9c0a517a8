"""FP64 CPU oracle for the LArTPC signal-simulation hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links or
executes this package: only tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP implementation.

Modules and what each follows (arXiv:2104.08265, Yu et al., "Evaluation of Portable
Acceleration Solutions for LArTPC Simulation Using Wire-Cell Toolkit"):

* ``raster``   - Sec. 2.1.1: the charge distribution S is built by rasterising each
                 deposition into a small patch and adding the patches into a large
                 grid ("rasterization" + "scatter adding").  Patch = truncated 2D
                 Gaussian integrated over (impact bin x tick) cells.
* ``convolve`` - Eq. 1 (signal term) and Eq. 2: M = R (*) S, a 2D convolution of the
                 arriving-charge distribution with the impulse response, evaluated by
                 its plain definition (direct sum) and by FFT in the frequency domain.
* ``fluct``    - Sec. 4.3.1 / Table 2: binomial fluctuation of the rasterised charge,
                 driven by a counter-based Philox4x32-10 stream (the RNG is factored out
                 of the main loop, Sec. 5) and an exact two-regime binomial sampler
                 that uses IEEE +,-,*,/ only.
* ``normal``   - Sec. 4.3.1 (the Kokkos port's Box-Muller transform): a fluctuation mode
                 that replaces each cell's binomial count by its normal approximation,
                 the normals drawn by Box-Muller from the binomial mode's Philox blocks.
* ``noise``    - Eq. 1's additive noise term N (Sec. 2): stationary noise per wire from
                 an amplitude spectrum and Philox-keyed complex normals, inverse real
                 transform along ticks.
* ``drift``    - Fig. 2 / Sec. 2.1.1: drift of 3D ionisation clouds to the readout, their
                 diffusion along and across the drift, attenuation by the electron
                 lifetime, and projection onto each plane's wire pitch and ticks.
* ``adc``      - Eq. 1 / Sec. 2: M as an ADC value; a linear converter per plane (gain,
                 pedestal, largest code), rounding half up, computed in a stated type.
* ``grad``     - adjoint of the convolution and per-deposition gradients of the
                 raster (differentiable mode; a reading beyond the paper, stated in
                 each function).

Pins (see tests/test_oracle_*.py): closed-form erf sums, charge conservation inside
the window, brute-force direct convolution, delta / shift responses, linearity,
padding invariance, adjoint identity, finite differences, the binomial law against
scipy.stats.binom, Philox against rocRAND's independent implementation, the Box-Muller
normals against libm and the normal law.
"""
