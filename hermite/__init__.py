"""4th-order Hermite integrator with individual block time steps, driving a
GRAPE-6-style force library: the client side of the paper's CPU/GPU split
(Sec. 2 and 2.1).  The i-particles are predicted and corrected on the host;
forces come from a backend (``G6Backend`` for libg6mi)."""

from .driver import HermiteState, BlockStepIntegrator, G6Backend, kepler_binary  # noqa: F401
