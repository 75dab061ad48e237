"""Plain FP64 CPU oracle for the Poisson-lognormal MAP filter (Kitaura, Jasche
& Metcalf, arXiv:0911.1407).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the test suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
implementation (no kernels, headers, helpers, tables or constant generators).

What it computes (every function cites the passage it follows):

* ``grid``      -- the periodic grid, Fourier-mode folding, prior eigenvalues
                   (section 2.2: S is a convolution, diagonal in Fourier space;
                   section 2.3: S_L likewise).
* ``dft``       -- the discrete Fourier transform written out as dense DFT
                   matrices (the definition), plus numpy's FFT as a library
                   primitive for grids too large for the dense form.
* ``model``     -- the negative log-posterior of the lognormal prior (section
                   2.3, log-prior equation) plus the Poisson likelihood
                   (section 2.1, eqs. 1-3) with the power-law bias of section
                   2.4; its gradient (section 3.1.2, gradient of the quadratic
                   form) and Hessian (section 3.1.2, Hessian).
* ``newton``    -- the Newton-Raphson iteration of section 3.1 in two forms:
                   a dense-Hessian Newton (Cholesky) for grids up to 16^3, and
                   an inexact Newton-Krylov iteration whose Krylov step length
                   is the step size of eq. (New5), with the iterate held as a
                   half-complex spectrum.
* ``adjoint``   -- the adjoint (implicit-function) derivative of a scalar
                   loss of the MAP field with respect to the model parameters.
* ``lambertw``  -- the principal branch of the Lambert W function by Halley's
                   iteration (Corless et al. 1996), for closed-form pins.
* ``gaussian``  -- the MAP of the Gaussian-prior model (section 2.2, unit
                   bias, eq. MAPG), the paper's comparison MAP filter.
* ``linbias``   -- the MAP with the linear (non-local) bias of sections
                   2.2.1 and 2.4.1, for the lognormal and the Gaussian prior.
* ``prior``     -- the lognormal prior covariance and mean built from a
                   matter spectrum (section 2.3, S_L(r) = ln(1 + S(r)),
                   mu = -S_L(0)/2).
* ``wiener``    -- the paper's comparison estimators (section 4.1.1: inverse
                   weighting and the LSQ-Wiener filter) and quality measures
                   (section 4.1.2: correlation coefficient, Euclidean
                   distance).
* ``closed_form`` -- closed-form MAP fields for special cases (white prior,
                   uniform data, zero completeness) and their derivatives.

Parity status: no function here is pinned to a value printed in the paper
(the paper prints no worked example; its figures carry no numbers in the
available text).  Each function is instead pinned by the mathematics: the
dense DFT against closed-form plane waves and the library FFT, the gradient
and Hessian against finite differences of the objective, the MAP against
dense Newton and against Lambert-W closed forms, the adjoint against central
finite differences and closed-form implicit derivatives.
"""
