"""The allocation-free apply (fnpf_laplace_apply_noalloc, called through the C ABI) against
fnpf_laplace_apply: the same kernels with the face slots in the library's static scratch array,
so the results must be bitwise identical.  Two calls in a row on one GPU, the second on a smaller
mesh (the scratch keeps the first call's contents, which the second must not see), FP64 and FP32,
with and without the Dirichlet mask; and the size limit is reported as an argument error."""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_09435_amd import fnpf
from workloads import configs


def _noalloc(ctx, x, y, mask):
    dt = fnpf.F64 if x.dtype == torch.float64 else fnpf.F32
    st = fnpf.lib().fnpf_laplace_apply_noalloc(ctx._h, dt, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                               int(mask), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_noalloc_apply_equals_apply_two_calls():
    big = configs.small_box(nx=7, ny=5, nz=3, p=6, periodic=(True, False), seed=3)    # 7 tiles, face slots
    small = configs.small_box(nx=4, ny=3, nz=2, p=4, periodic=(False, True), seed=4)  # smaller input
    g = torch.Generator(device="cuda").manual_seed(0)
    for wl in (big, small):
        s = fnpf.setup_workload(wl, fp32=True)
        s.ctx.geom(s.eta0, s.h)
        for dtype in (torch.float64, torch.float32):
            x = torch.randn(wl.mesh.n_v, dtype=torch.float64, device="cuda", generator=g).to(dtype)
            for mask in (0, 1):
                ref = s.ctx.laplace_apply(x, mask_dirichlet=bool(mask))
                y = torch.full_like(x, float("nan"))
                assert _noalloc(s.ctx, x, y, mask) == 0, fnpf.lib().fnpf_last_error(s.ctx._h)
                torch.cuda.synchronize()
                assert torch.equal(y, ref), (wl.mesh.n_v, dtype, mask)
        s.ctx.close()


def test_noalloc_apply_rejects_meshes_beyond_its_scratch():
    # degree 1 with 100 layers: 101 node levels of face slots between the 64-column tiles of a
    # 600 x 600 grid need more than the 128 MiB scratch in FP64
    from workloads import mesh as wm
    m = wm.structured_box(600, 600, 0.0, 1.0, 0.0, 1.0, False, False, p=1, nz=100)
    ctx = fnpf.Context(m)
    z = torch.zeros(m.n_s, dtype=torch.float64, device="cuda")
    ctx.geom(z, z + 1.0)
    x = torch.zeros(m.n_v, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    assert _noalloc(ctx, x, y, 0) == 1                       # FNPF_ERR_ARG
    assert b"scratch" in fnpf.lib().fnpf_last_error(ctx._h)
    ctx.close()
