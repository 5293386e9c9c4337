"""The allocation-free learned-beam loss / gradient entry point against the allocating one.

matvis_mlp_loss_grad_noalloc runs the same kernels as matvis_mlp_loss_grad on a
workspace carved from a fixed device array instead of hipMalloc'd buffers.  Both
are called through the C ABI on the same seeded inputs, twice in a row (the
second call with fewer rows, on the workspace the first call left behind), in
the bf16 product mode and the FP32 check mode; the outputs must agree to the
learned beam's FP32 gradient bar (1e-5 relative, normwise), and in practice
bitwise.  Sizes above the fixed workspace are rejected.
"""
import ctypes

import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    import torch
    from paper_2312_09763_amd import synth
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    y = rng.normal(0.0, 0.3, (n, 8)).astype(np.float32)
    p = synth.surrogate_init(seed)
    return (torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())


@pytest.mark.parametrize("fp32_math", [False, True])
def test_noalloc_matches_allocating_entry_point(fp32_math):
    import torch
    from paper_2312_09763_amd import matvis as mv
    torch.cuda.set_device(0)
    for call, n in enumerate((3000, 700)):  # second call smaller, ragged against the 256-row blocks
        say(f"no-alloc loss/grad: call {call}, n={n}, fp32_math={fp32_math}")
        params, x, y = _inputs(n, 11 + call)
        g_ref, l_ref = mv.mlp_loss_grad(params, x, y, fp32_math=fp32_math)
        grad = torch.full_like(params, float("nan"))
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        mv.mlp_loss_grad_noalloc(params, x, y, grad, loss, fp32_math=fp32_math)
        torch.cuda.synchronize()
        g, gr = grad.cpu().numpy().astype(np.float64), g_ref.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(g))
        rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
        say(f"  grad rel diff {rel:.3e} (bitwise equal: {np.array_equal(g, gr)}), loss {loss.item():.6e} vs "
            f"{l_ref.item():.6e}")
        assert rel <= 1e-5
        assert abs(loss.item() - l_ref.item()) <= 1e-6 * abs(l_ref.item())


def test_noalloc_size_limit():
    import torch
    from paper_2312_09763_amd import matvis as mv
    L = mv.load_library()
    torch.cuda.set_device(0)
    for n, want in ((4096, mv.OK), (4097, mv.EINVAL)):
        say(f"no-alloc size limit: n={n}")
        params, x, y = _inputs(n, 5)
        grad = torch.empty_like(params)
        loss = torch.empty((1,), dtype=torch.float32, device="cuda")
        st = L.matvis_mlp_loss_grad_noalloc(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(y.data_ptr()), n, 0, ctypes.c_void_p(grad.data_ptr()),
                                            ctypes.c_void_p(loss.data_ptr()), None)
        torch.cuda.synchronize()
        assert st == want, (n, st)
        if st == mv.OK:
            g_ref, l_ref = mv.mlp_loss_grad(params, x, y)
            assert torch.equal(grad, g_ref) or float((grad - g_ref).norm() / g_ref.norm()) <= 1e-5
