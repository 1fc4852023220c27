"""Several operands in one arrow_spmm call: operands of one storage type and
tile width share one launch sequence (the matrix is read once for all of
them), and every operand's result is bitwise the one it gets alone."""
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


def _operand(plan, x_plan, k, dtype, t):
    """Buffers of one operand whose input is x_plan (a step t > 0 folds a 1/nu)."""
    dev = "cuda"
    scaled = dtype in ("f16", "f8e4m3")
    y = plan.empty(k, dtype)
    st = dict(y=y, nrm=torch.zeros(k, dtype=torch.float64, device=dev),
              inv=torch.zeros(k, dtype=torch.float64, device=dev),
              xinv=torch.full((k,), 0.5, dtype=torch.float64, device=dev),
              xs=torch.ones(k, dtype=torch.float32, device=dev),
              xm=torch.full((k,), 448.0, dtype=torch.float32, device=dev),
              ys=torch.ones(k, dtype=torch.float32, device=dev),
              ym=torch.zeros(k, dtype=torch.float32, device=dev))
    op = A_.operand(x_plan, y, dtype, x_scale=st["xs"] if scaled else None,
                    x_inv_norm=st["xinv"] if t > 0 else None,
                    x_maxabs=st["xm"] if scaled else None,
                    y_scale=st["ys"] if scaled else None, y_maxabs=st["ym"] if scaled else None,
                    y_norm=st["nrm"], y_inv_norm=st["inv"])
    return op, st


@pytest.mark.parametrize("graph", ["rmat13", "grid3d20"])
def test_operands_share_launches_and_match_alone(graph):
    if graph == "rmat13":
        M, b = W.make_matrix("rmat", 13, "row_normalized", 61, 62, 16), 128
    else:
        M, b = W.make_matrix("grid3d", 20, "sym_laplacian", 63, 64), 400
    d = A_.Decomposition.from_matrix(M, b, seed=5)
    plan = A_.Plan(d)
    vop0 = d.level(0)["vop"].astype(np.int64)
    # (k, dtype, step): five tile-width-16 operands (one launch sequence), a
    # k=32 FP32 operand and two BF16 operands (their own sequences)
    specs = [(16, "f32", 0), (48, "f32", 1), (80, "f32", 0), (16, "f32", 1), (112, "f32", 0),
             (32, "f32", 0), (64, "bf16", 0), (64, "bf16", 1)]
    xs = []
    for i, (k, dtype, t) in enumerate(specs):
        X0 = W.features(M.n, k, 700 + i)
        xp = plan.empty(k, dtype)
        plan.permute_in(torch.from_numpy(X0).cuda(), xp, dtype)
        xs.append((X0, xp))
    # alone, one call per operand
    alone = []
    for (k, dtype, t), (X0, xp) in zip(specs, xs):
        op, st = _operand(plan, xp, k, dtype, t)
        plan.spmm([op], plan.workspace(plan.workspace_size(k, dtype)))
        alone.append(st)
    torch.cuda.synchronize()
    # together, one call
    ops, sts, total = [], [], 0
    for (k, dtype, t), (X0, xp) in zip(specs, xs):
        op, st = _operand(plan, xp, k, dtype, t)
        ops.append(op)
        sts.append(st)
        total += plan.workspace_size(k, dtype)
    ws = plan.workspace(total)
    plan.profile(True)
    plan.spmm(ops, ws)
    torch.cuda.synchronize()
    launches = plan.profile_query(A_.KERNEL_LEVEL0)[0]
    plan.profile(False)
    # tile width 16: 1+3+5+1+7 = 17 tiles -> 3 launches of <= 8 tiles;
    # tile width 32: 1; BF16 tile width 64: 2 tiles -> 1
    say(f"[batch] {graph}: {len(specs)} operands in {launches} level-0 launches")
    assert launches == 5
    for i, ((k, dtype, t), a, m) in enumerate(zip(specs, alone, sts)):
        assert torch.equal(a["y"].view(torch.uint8), m["y"].view(torch.uint8)), i
        assert torch.equal(a["nrm"], m["nrm"]) and torch.equal(a["inv"], m["inv"]), i
        if dtype == "f32":
            X0 = xs[i][0].astype(np.float64) * (0.5 if t > 0 else 1.0)
            y = np.empty((M.n, k))
            y[vop0] = m["y"].cpu().numpy()
            assert S.rel_fro(y, S.csr_spmm(M, X0)) <= 1e-5, i
    # an operand may not write what another one reads
    op0, _ = _operand(plan, xs[0][1], 16, "f32", 0)
    op1 = A_.operand(sts[3]["y"], xs[0][1], "f32")  # op1 writes op0's input
    with pytest.raises(A_.ArrowError):
        plan.spmm([op0, op1], plan.workspace(2 * plan.workspace_size(16)))
