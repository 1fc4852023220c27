"""The allocation-free entry point arrow_spmm_static against arrow_spmm
(caller workspace): the same products bit for bit, on two calls in a row, the
second with a smaller input; sizes beyond the fixed workspace are refused
before any device work."""
import numpy as np
import pytest

import workloads as W
from oracle import spmm as S
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


def _plan(M, b, seed):
    d = A_.Decomposition.from_matrix(M, b, seed=seed)
    return A_.Plan(d), d.level(0)["vop"].astype(np.int64)


def _one(plan, vop0, M, k, dtype, x_seed):
    """One product through both entry points; returns (y_ws, y_static, norms...)."""
    X0 = W.features(M.n, k, x_seed)
    x = torch.from_numpy(X0).cuda()
    xp = plan.empty(k, dtype)
    scaled = dtype in ("f16", "f8e4m3")
    xs = torch.ones(k, dtype=torch.float32, device="cuda")
    xm = torch.zeros(k, dtype=torch.float32, device="cuda")
    plan.permute_in(x, xp, dtype, x_scale=xs if scaled else None,
                    x_maxabs=xm if scaled else None)
    outs = []
    for static in (False, True):
        y = plan.empty(k, dtype)
        y.fill_(0)
        nrm = torch.full((k,), -1.0, dtype=torch.float64, device="cuda")
        inv = torch.full((k,), -1.0, dtype=torch.float64, device="cuda")
        ysc = torch.zeros(k, dtype=torch.float32, device="cuda")
        ymx = torch.zeros(k, dtype=torch.float32, device="cuda")
        op = A_.operand(xp, y, dtype, x_scale=xs if scaled else None,
                        x_maxabs=xm if scaled else None,
                        y_scale=ysc if scaled else None, y_maxabs=ymx if scaled else None,
                        y_norm=nrm, y_inv_norm=inv)
        if static:
            plan.spmm_static([op])
        else:
            ws = plan.workspace(plan.workspace_size(k, dtype))
            plan.spmm([op], ws)
        torch.cuda.synchronize()
        outs.append((y, nrm, inv, ysc))
    return X0, xp, outs


def _compare(label, plan, vop0, M, k, dtype, x_seed):
    X0, xp, ((y0, n0, i0, s0), (y1, n1, i1, s1)) = _one(plan, vop0, M, k, dtype, x_seed)
    ws_need = plan.workspace_size(k, dtype)
    say(f"[no-alloc] {label}: n={M.n} nnz={M.nnz} k={k} {dtype} workspace {ws_need} bytes")
    assert ws_need <= A_.STATIC_WORKSPACE_BYTES
    # bit for bit the same as the caller-workspace entry point
    assert torch.equal(y0.view(torch.uint8), y1.view(torch.uint8))
    assert torch.equal(n0, n1) and torch.equal(i0, i1) and torch.equal(s0, s1)
    if dtype == "f32":
        # and within the FP32 bar of the FP64 oracle
        y = np.empty((M.n, k))
        y[vop0] = y1.cpu().numpy()
        assert S.rel_fro(y, S.csr_spmm(M, X0.astype(np.float64))) <= 1e-5


def test_static_matches_caller_workspace_twice_then_smaller():
    # first call: a multi-level R-MAT with hub chunks and upper-pass rows
    # (partial rows in the workspace), k = 64
    R = W.make_matrix("rmat", 13, "row_normalized", 41, 42, 16)
    plan_r, vop_r = _plan(R, 64, 3)
    info = plan_r.info()
    assert info["chunks"] > 0 and info["levels"] > 1
    _compare("rmat13 k=64", plan_r, vop_r, R, 64, "f32", 5)
    # second call: a smaller input on another plan (fewer rows, fewer columns)
    G = W.make_matrix("grid2d", 40, "uniform", 43, 44)
    plan_g, vop_g = _plan(G, 40, 4)
    _compare("grid40 k=16", plan_g, vop_g, G, 16, "f32", 6)
    # and the first plan again with a narrower operand and a scaled format
    _compare("rmat13 k=32 f8", plan_r, vop_r, R, 32, "f8e4m3", 7)
    _compare("rmat13 k=16 bf16", plan_r, vop_r, R, 16, "bf16", 8)


def test_static_refuses_oversize_before_device_work():
    R = W.make_matrix("rmat", 12, "row_normalized", 45, 46, 16)
    plan, _ = _plan(R, 64, 5)
    # the smallest k (multiple of 16) whose workspace exceeds the fixed array
    k = 16
    while plan.workspace_size(k) <= A_.STATIC_WORKSPACE_BYTES:
        k *= 2
    # never dereferenced: the size check comes before any device work
    fake = 1 << 44
    op = A_.Operand(fake, fake * 2, k, k, k, A_.F32, 0, None, None, None, None, None, None, None)
    with pytest.raises(A_.ArrowError) as e:
        plan.spmm_static([op])
    assert e.value.status == A_.ERR_UNSUPPORTED
    assert "static workspace" in A_.lib().arrow_last_error().decode()
    # the entry point still works afterwards
    G = W.make_matrix("grid2d", 16, "uniform", 47, 48)
    plan_g, vop_g = _plan(G, 16, 6)
    _compare("grid16 k=16 after refusal", plan_g, vop_g, G, 16, "f32", 9)
