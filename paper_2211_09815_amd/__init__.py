"""MI355X particle-mesh hot path of the adjoint-method differentiable
simulation: libpm.so (HIP kernels behind include/pm.h) and its thin Python
binding.

    from paper_2211_09815_amd import api, force, force_vjp, Simulate
"""
from .autograd import force, force_vjp  # noqa: F401
from .simulate import Simulate, SimConfig, Simulation  # noqa: F401
