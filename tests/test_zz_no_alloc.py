"""cpdnet_forward_noalloc against cpdnet_forward.

The no-allocation entry point runs the same network kernels with the
library's static device scratch in place of a caller workspace, so its W0
must equal the workspace entry point's bit for bit.  Two calls in a row, the
second on smaller sets, show that nothing left in the scratch by the first
call leaks into the second; a size beyond the scratch is refused before any
device work."""
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _pair(lib, batch, M, N, seed):
    X, _, _ = lib.synth_pairs(batch, M, beta=2.0, coef=0.1, seed0=seed)
    _, Y, _ = lib.synth_pairs(batch, N, beta=2.0, coef=0.1, seed0=seed + 7919)
    return X.contiguous(), Y.contiguous()


def test_noalloc_forward_equals_workspace_forward(lib):
    import torch
    net = lib.WarmStartNet(seed=5, out_scale=1.0)
    for batch, M, N, seed in ((3, 1500, 1700, 11), (1, 700, 500, 29)):
        say("noalloc forward", batch, M, N, seed)
        X, Y = _pair(lib, batch, M, N, seed)
        ref = net.forward(X, Y)
        out = net.forward_noalloc(X, Y)
        torch.cuda.synchronize()
        assert torch.isfinite(ref).all()
        assert float(ref.abs().max()) > 0.0
        assert torch.equal(out, ref), float((out - ref).abs().max())


def test_noalloc_forward_refuses_sizes_beyond_the_scratch(lib):
    import ctypes
    import torch
    net = lib.WarmStartNet(seed=5)
    n = ctypes.c_size_t(0)
    lib._check(lib.load_library().cpdnet_workspace_size(8, 2000, 2000, lib.CPDNET_BF16,
                                                        ctypes.byref(n)))
    assert n.value > 64 << 20
    X = torch.zeros(8, 2000, 3, device="cuda")
    with pytest.raises(lib.FastCPDError) as e:
        net.forward_noalloc(X, X)
    assert e.value.status == lib.CPD_E_WORKSPACE
