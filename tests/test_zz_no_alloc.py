"""lddmm_bl_project_noalloc, the projection for callers that cannot allocate device memory, against
lddmm_bl_project: the same kernels with the reduction's workspace in the library's static device array,
so the two results agree bit for bit (and within the FP32 projection tolerance 1e-6 of the oracle
checks).  Two calls in a row on different contexts, the second with a smaller input, check that the
shared array carries nothing from one call to the next; sizes beyond the array and contexts off the
plane-wise FP32 path are rejected with an error."""
import numpy as np
import pytest
import torch

from gpu_common import close
from paper_2006_06823_amd import lddmm_bl as L

pytestmark = pytest.mark.gpu


def _grid(ctx, ncomp, seed):
    g = torch.Generator().manual_seed(seed)
    shape = ctx._grid_shape(ncomp if ncomp > 1 else None)
    return torch.rand(shape, generator=g, dtype=torch.float32).to("cuda") - 0.5


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_projection_equals_projection(order):
    cases = [((64, 48, 40), (16, 12, 16), 4, 11), ((32, 24, 20), (8, 8, 6), 1, 12)]
    for n, k, ncomp, seed in cases:
        print(f"[no-alloc] grid {n} band {k} ncomp {ncomp}", flush=True)
        ctx = L.Context(L.Problem(n, k, nt=2, variant=L.IMAGE_TRANSPORT, precision=L.FP32))
        f = _grid(ctx, ncomp, seed)
        ref = ctx.project(f, ncomp)
        out = ctx.empty_bl(ncomp if ncomp > 1 else None).fill_(float("nan"))
        ctx.project_noalloc(f, out, ncomp)
        ctx.stream.synchronize()
        assert torch.equal(out, ref), "static-workspace projection differs from the context-workspace one"
        assert close(out, ref, f"no-alloc vs project {n}") <= 1e-6
        ctx.close()


def test_noalloc_rejects_oversized_and_fp64():
    ctx = L.Context(L.Problem((96, 96, 96), (64, 64, 64), nt=1, variant=L.IMAGE_TRANSPORT, precision=L.FP32))
    f = torch.zeros((12, 96, 96, 96), dtype=torch.float32, device="cuda")
    out = ctx.empty_bl(12)
    with pytest.raises(L.LddmmError) as e:
        ctx.project_noalloc(f, out, 12)
    assert e.value.status == -1 and "static scratch" in str(e.value)
    ctx.close()
    ctx = L.Context(L.Problem((24, 20, 28), (8, 8, 10), nt=1, variant=L.IMAGE_TRANSPORT, precision=L.FP64))
    f = torch.zeros((24, 20, 28), dtype=torch.float64, device="cuda")
    with pytest.raises(L.LddmmError) as e:
        ctx.project_noalloc(f, ctx.empty_bl(), 1)
    assert e.value.status == -1
    ctx.close()
