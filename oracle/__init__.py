"""FP64 CPU oracle for the batched differentiable quadrotor environment step.

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
HIP path is checked against. Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product library never does,
and it shares no code with the HIP kernels or their host layer.

Everything is written with plain torch CPU ops in float64, vectorised over
agents / rays / primitives, with no blocking, fusion or reordering beyond the
definitions. Where the paper fixes the arithmetic (Sec. III-A, Eqs. 1-5;
Sec. III-B ray casting against primitives) the oracle writes that definition
out; derivatives are taken with torch autograd (a library primitive that
differentiates exactly what is written), which the CPU tests pin against
central finite differences with frozen hit topology.

Modules:
  dynamics   point-mass (Eq. 3), full rigid body (Eq. 1 + body-rate loop),
             nominal (Eq. 2) models; Euler and RK4
  sensors    camera / LiDAR ray generation, brute-force ray casting against
             spheres, boxes, agent spheres and the room, collisions
  policy     the MLP policy, observation, loss and BPTT over a rollout (Eq. 5)
  surrogate  BF16-rounded residual MLP, MSE, Adam, surrogate step + judge
"""
from . import dynamics, sensors, policy, surrogate  # noqa: F401
