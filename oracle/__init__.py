"""CPU oracle for the finite-volume + immersed-boundary time step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never calls it and shares no code with it.

It is a plain, slow, float64 implementation written from the paper
(Fan, Liu, Wang & Wang, "Diff-FlowFSI", arXiv 2505.23940), Sec. 2.3:

* fluid  (``fluid.py``)  -- staggered finite volumes, central / upwind
  convection in divergence form, central diffusion, forward-Euler predictor
  (Eq. 4), direct forcing (Eq. 5), modified pressure Poisson equation
  (Eq. 9) and velocity correction (Eq. 10);
* Poisson (``poisson.py``) -- the exact solution of the discrete PPE by
  tensor-product eigen-decomposition (the plain definition the GPU reaches
  iteratively);
* IBM   (``ibm.py``)    -- solid / immersed-boundary point classes
  (Sec. 2.2, Fig. 2), solid-to-fluid interpolation (Eqs. 18-19) and
  fluid-to-solid spreading (Eq. 20) with the 4-point kernel (Eqs. 21-22);
* body  (``body.py``)   -- rigid spring-damper oscillator with classic RK4
  (Eq. 12);
* LES   (``les.py``)    -- constant Smagorinsky subgrid stress and the
  equilibrium wall-stress model with the Spalding law (Sec. 3.4.5,
  Eqs. 27-29), added to the momentum right-hand side;
* step  (``step.py``)   -- one weakly coupled step (Alg. 1 with N = 1),
  rollouts and the two loss functionals.

The discrete adjoint of the oracle is ``torch.autograd`` over these float64
operations with the masks detached (the masks are piecewise constant in the
body position, so their derivative is zero).

Where the paper is silent or ambiguous, the reading taken is stated in the
docstring of the function that implements it.
"""
from .grid import Grid  # noqa: F401
from .step import step, rollout, init_state, make_params  # noqa: F401
