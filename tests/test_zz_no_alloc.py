"""helm_vcycle_noalloc (the cycle without allocation: level vectors in the
library's per-device scratch array) against helm_vcycle (the same cycle in
a caller workspace), through the C ABI: bit-identical results on 2D and 3D
meshes in both precision modes, two calls in a row with the second on a
smaller input, and the size limit reported as an error that leaves the
entry point usable."""

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

DT = {"fp64": "complex128", "fp32": "complex64"}


def _solver(dim, n, levels, k, prec):
    from paper_2506_18694_amd import Solver
    return Solver(dim, n, levels, k, 0.0, k, precision=prec)


def _rand(nrhs, N, seed, prec):
    return to_dev(W.random_complex((nrhs, N), seed), DT[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_workspace_cycle_2d(prec):
    s = _solver(2, 512, 7, 51.2, prec)
    # first call: no height measured yet on this mesh (model heights), two columns
    b2 = _rand(2, s.N, 61, prec)
    x_na = s.vcycle_noalloc(b2)
    x_ws = s.vcycle(b2)
    torch.cuda.synchronize()
    assert torch.equal(x_na, x_ws)
    assert torch.isfinite(torch.view_as_real(x_na)).all()
    # second call, smaller input: one column on the same handle
    b1 = _rand(1, s.N, 62, prec)
    x_na1 = s.vcycle_noalloc(b1)
    torch.cuda.synchronize()
    assert torch.equal(x_na1, s.vcycle(b1))
    s.close()
    # a smaller mesh on another handle shares the same scratch
    t = _solver(2, 64, 3, 10.0, prec)
    c = _rand(1, t.N, 63, prec)
    y = t.vcycle_noalloc(c)
    torch.cuda.synchronize()
    assert torch.equal(y, t.vcycle(c))
    t.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_workspace_cycle_3d(prec):
    s = _solver(3, 64, 4, 20.0, prec)
    b = _rand(2, s.N, 64, prec)
    x_na = s.vcycle_noalloc(b)
    torch.cuda.synchronize()
    assert torch.equal(x_na, s.vcycle(b))
    b1 = _rand(1, s.N, 65, prec)
    x1 = s.vcycle_noalloc(b1)
    torch.cuda.synchronize()
    assert torch.equal(x1, s.vcycle(b1))
    s.close()


def test_noalloc_rejects_oversize_and_stays_usable():
    from paper_2506_18694_amd import helm
    s = _solver(2, 1024, 8, 100.0, "fp64")
    b = _rand(4, s.N, 66, "fp64")  # 4 columns of 1025^2 FP64 values exceed 64 MiB
    with pytest.raises(helm.HelmError) as ei:
        s.vcycle_noalloc(b)
    assert ei.value.status == helm.HELM_EINVAL
    assert "bytes of scratch" in str(ei.value)
    b1 = b[:1].contiguous()
    x1 = s.vcycle_noalloc(b1)
    torch.cuda.synchronize()
    assert torch.equal(x1, s.vcycle(b1))
    s.close()
