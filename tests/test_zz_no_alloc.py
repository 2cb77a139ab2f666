"""policy_forward_noalloc (the policy forward for callers that cannot allocate
device memory) against policy_forward through the C ABI: the same kernels on
scratch in a fixed device array instead of a per-call allocation, so the
outputs must be equal bit for bit; two calls in a row, the second on a
smaller batch, so that stale scratch of the first call cannot leak into the
second; sizes above the scratch limit are refused with an error."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import policy as opol
from tests.helpers import cuda, f64, print_case

pytestmark = pytest.mark.gpu

FP32, X3 = 0, 1  # POLICY_GEMM_FP32, POLICY_GEMM_BF16X3
MAX_B = 512      # POLICY_NOALLOC_MAX_B


def _inputs(rng, B):
    x = rng.uniform(0, 1, (B, 3081)).astype(np.float32)
    x[:, 3072:] = rng.normal(size=(B, 9))
    return x


@pytest.mark.parametrize("mode", [FP32, X3])
def test_noalloc_forward_equals_policy_forward(mode):
    from paper_2509_10247_amd import _lib
    rng = np.random.default_rng(90 + mode)
    theta = wl.flatten_mlp(wl.mlp_init(rng, wl.POLICY_DIMS))
    th = cuda(theta)
    thd = opol.unflatten(torch.tensor(theta.astype(np.float64)), wl.POLICY_DIMS)
    for B in (MAX_B, 300, 77):  # the limit itself, then smaller batches with a ragged tail
        print_case("noalloc_forward", B=B, gemm=mode)
        x = cuda(_inputs(rng, B))
        y_ref = torch.empty(B, 4, device="cuda")
        _lib.policy_forward(th, x, y_ref, mode)
        y = torch.full((B, 4), float("nan"), device="cuda")
        _lib.policy_forward_noalloc(th, x, y, mode)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), f"B={B}: differs from policy_forward"
        yo = opol.mlp_tanh(thd, f64(x))
        assert (f64(y) - yo).abs().max() < 2e-5


def test_noalloc_forward_rejects_oversized_batch():
    from paper_2509_10247_amd import _lib
    th = torch.zeros(855812, device="cuda")
    x = torch.zeros(MAX_B + 1, 3081, device="cuda")
    y = torch.zeros(MAX_B + 1, 4, device="cuda")
    with pytest.raises(RuntimeError, match="scratch limit"):
        _lib.policy_forward_noalloc(th, x, y, FP32)
    e = torch.zeros(0, 3081, device="cuda")
    _lib.policy_forward_noalloc(th, e, torch.zeros(0, 4, device="cuda"), FP32)
