"""mbp_residual_norm_noalloc (the check that allocates nothing) against
mbp_residual_norm, through the C ABI: two calls in a row, the second on a
smaller problem, both compared with the allocating entry point's result and
with the oracle's residual norm; a problem whose partial sums exceed the
fixed scratch array is refused with MBP_ERR_TOO_LARGE."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def mbp():
    import paper_2106_03583_amd as m
    return m


def _call(mbp, fn, plan, f, p, shift, out):
    stream = C.c_void_p(__import__("torch").cuda.current_stream().cuda_stream)
    return fn(plan.handle, C.c_void_p(f.data_ptr()), C.c_void_p(p.data_ptr()), C.c_double(shift),
              C.c_void_p(out.data_ptr()), stream)


def test_noalloc_matches_allocating_entry_point(torch_cuda, mbp):
    torch = torch_cuda
    cases = [(W.lshape(64, 24, 1.5, 1.0), 0.0, 0.25),   # larger first
             (W.box(40, 30, 6, 0.5, 0.4, 0.1, "DD", "PP", "ND", xfactor=1.4, name="small"), 3.5, 0.0)]
    assert mbp.lib.mbp_noalloc_scratch_bytes() == 8 << 20
    for prob, alpha, shift in cases:
        print(f"no-alloc check {prob.name} alpha={alpha}", flush=True)
        rng = np.random.default_rng(81)
        f = rng.standard_normal(prob.ncells)
        p = rng.standard_normal(prob.ncells)
        fd = torch.from_numpy(f).cuda()
        pd = torch.from_numpy(p).cuda()
        plan = mbp.Plan(prob, helmholtz=alpha)
        a = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
        b = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
        assert _call(mbp, mbp.lib.mbp_residual_norm, plan, fd, pd, shift, a) == mbp.OK
        assert _call(mbp, mbp.lib.mbp_residual_norm_noalloc, plan, fd, pd, shift, b) == mbp.OK
        torch.cuda.synchronize()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        r = f - shift - oracle.apply_3d(oracle.Geometry(prob), p, alpha)
        ref = np.array([np.linalg.norm(r), np.linalg.norm(f - shift)])
        print(f"  allocating {a}  no-alloc {b}  oracle {ref}", flush=True)
        assert np.allclose(b, a, rtol=1e-14, atol=0.0)
        assert np.allclose(b, ref, rtol=1e-12, atol=0.0)
        plan.close()


def test_noalloc_refuses_too_large(torch_cuda, mbp):
    torch = torch_cuda
    # 16 * nz * tiles bytes of partial sums: a row of 250 joined 4 x 4 blocks
    # (one 64 x 16 tile each) and 2200 z cells need 8.8 MB > 8 MiB
    nb, n = 250, 4
    blocks = []
    for i in range(nb):
        bc = (W.DIRICHLET if i == 0 else W.CONNECT, W.DIRICHLET if i == nb - 1 else W.CONNECT,
              W.NEUMANN, W.NEUMANN)
        blocks.append(W.Block((n * i + 1, 1), (n * i + n, n), W.faces(n, float(i), float(i + 1)),
                              W.faces(n, 0.0, 1.0), bc))
    prob = W.Problem(blocks, 2200, 1.0, W.PAIRS["PP"], name="too_large")
    plan = mbp.Plan(prob)
    f = torch.zeros(prob.ncells, dtype=torch.float64, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    assert _call(mbp, mbp.lib.mbp_residual_norm_noalloc, plan, f, f, 0.0, out) == mbp.ERR_TOO_LARGE
    plan.close()
