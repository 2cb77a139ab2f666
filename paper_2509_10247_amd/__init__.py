"""MI355X-native batched, differentiable quadrotor environment step.

The compute lives in libdiffaero.so (hand-written HIP kernels for gfx950
behind a C ABI, declared in include/diffaero.h). This package is the thin
Python side: `_lib` marshals arguments to the C entry points, `env` keeps a
simulator handle together with the device buffers it references, `bptt`
wraps the rollout gradient in a torch.autograd.Function, and `build`
compiles the library.
"""
__all__ = ["_lib", "env", "bptt", "build"]
