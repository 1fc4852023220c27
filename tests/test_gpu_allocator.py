"""Plan buffers through the allocator hook (arrow_set_allocator): every byte
of a plan comes from the installed allocator and goes back through it, and a
plan from PyTorch's caching allocator computes the same products bit for bit
as one from hipMalloc."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import say

torch = pytest.importorskip("torch")
A_ = pytest.importorskip("paper_2402_19364_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    A_.set_allocator(None, None)


def _product(plan, M, k):
    X0 = W.features(M.n, k, 11)
    x = torch.from_numpy(X0).cuda()
    xp = plan.empty(k)
    plan.permute_in(x, xp)
    y = plan.empty(k)
    nrm = torch.zeros(k, dtype=torch.float64, device="cuda")
    plan.spmm([A_.operand(xp, y, y_norm=nrm)], plan.workspace(plan.workspace_size(k)))
    torch.cuda.synchronize()
    return y.clone(), nrm.clone()


def test_allocator_hook_counts_every_plan_byte():
    M = W.make_matrix("rmat", 13, "row_normalized", 51, 52, 16)
    d = A_.Decomposition.from_matrix(M, 64, seed=2)
    ref_plan = A_.Plan(d)            # default allocator (hipMalloc)
    y_ref, n_ref = _product(ref_plan, M, 32)
    ref_plan.close()

    allocs, frees = [], []

    def alloc(nbytes, stream):
        p = torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), stream)
        allocs.append((p, nbytes))
        return p

    def free(p):
        frees.append(p)
        torch.cuda.caching_allocator_delete(p)

    A_.set_allocator(alloc, free)
    try:
        before = torch.cuda.memory_allocated()
        plan = A_.Plan(d)
        grew = torch.cuda.memory_allocated() - before
        fp = plan.footprint()
        say(f"[alloc] plan footprint {fp} bytes in {len(allocs)} allocations; "
            f"torch pool grew by {grew}")
        assert fp > 0 and sum(nb for _, nb in allocs) == fp
        assert grew >= fp                       # the bytes came from torch's pool
        assert all(p % 256 == 0 for p, _ in allocs)
        y, nrm = _product(plan, M, 32)
        assert torch.equal(y, y_ref) and torch.equal(nrm, n_ref)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated()
        plan.close()
        assert sorted(frees) == sorted(p for p, _ in allocs)
        # every plan byte went back to the pool (the product's tensors stay)
        assert held - torch.cuda.memory_allocated() == grew
        # the PyTorch allocator as packaged by the binding
        A_.use_torch_allocator()
        plan2 = A_.Plan(d)
        y2, n2 = _product(plan2, M, 32)
        assert torch.equal(y2, y_ref) and torch.equal(n2, n_ref)
        plan2.close()
    finally:
        A_.set_allocator(None, None)
    # a failing allocator is reported as out of memory, nothing leaks
    A_.set_allocator(lambda nbytes, stream: 0, lambda p: None)
    try:
        with pytest.raises(A_.ArrowError) as e:
            A_.Plan(d)
        assert e.value.status == A_.ERR_OUT_OF_MEMORY
    finally:
        A_.set_allocator(None, None)
