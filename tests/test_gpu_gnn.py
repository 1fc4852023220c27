"""The GNN-style step y = ReLU((A x) W) (Section 2: the iteration with an
element-wise sigma; here after a k x k weight matrix), fused into the level-0
pass on FP32 matrix cores, against the oracle's FP64 ReLU((A X) W).

Bound: FP32 accumulation of the sparse product (about deg * 2^-24 relative)
plus the FP32 k x k product on matrix cores (about k * 2^-24 relative); ReLU
is 1-Lipschitz.  Every step is gated at 1e-5 relative Frobenius error
(teacher-forced: the oracle takes exactly the x the GPU consumed)."""
import numpy as np
import pytest

import workloads as W
from oracle import spmm as S
from tests.gpu_helpers import say

torch = pytest.importorskip("torch")
A_ = pytest.importorskip("paper_2402_19364_amd")

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _graphs():
    return [
        ("grid64", W.workload_matrix(W.WORKLOADS["grid64"]), 64),
        # multi-level with hub rows (chunk and upper passes, listed partial rows)
        ("rmat12", W.make_matrix("rmat", 12, "row_normalized", 71, 72, 16), 64),
        # b > 21845: int32 columns in the level-0 pass
        ("rmat13_wide_b", W.make_matrix("rmat", 13, "row_normalized", 73, 74, 8), 22000),
    ]


def _to_orig(v_plan, vop0):
    out = np.empty_like(v_plan)
    out[vop0] = v_plan
    return out


@pytest.mark.parametrize("k", [16, 32, 64, 128])
def test_gnn_steps_match_oracle(k):
    for name, M, b in _graphs():
        d = A_.Decomposition.from_matrix(M, b, seed=3)
        plan = A_.Plan(d)
        vop0 = d.level(0)["vop"].astype(np.int64)
        rng = np.random.default_rng(k)
        Wm = (rng.standard_normal((k, k)) / np.sqrt(k)).astype(np.float32)
        w = torch.from_numpy(Wm).cuda()
        X = W.features(M.n, k, 900 + k)
        xp = plan.empty(k)
        plan.permute_in(torch.from_numpy(X).cuda(), xp)
        x_in = X.astype(np.float64)
        ws = plan.workspace(plan.workspace_size(k))
        for t in range(3):
            y = plan.empty(k)
            nrm = torch.zeros(k, dtype=torch.float64, device="cuda")
            plan.spmm([A_.operand(xp, y, w=w, y_norm=nrm)], ws)
            torch.cuda.synchronize()
            z = _to_orig(y.cpu().numpy().astype(np.float64), vop0)
            ref = S.gnn_layer(M, x_in, Wm)
            err = S.rel_fro(z, ref)
            num = np.sqrt(np.sum((z - ref) ** 2, axis=0))
            den = np.sqrt(np.sum(ref * ref, axis=0))
            col = float(np.max(np.where(den > 0, num / np.where(den > 0, den, 1), num)))
            nerr = float(np.max(np.abs(nrm.cpu().numpy() - np.sqrt(np.sum(z * z, axis=0))) /
                                np.maximum(np.sqrt(np.sum(z * z, axis=0)), 1e-300)))
            say(f"[gnn] {name} k={k} t={t}: rel {err:.2e}, worst column {col:.2e}, "
                f"norm of stored {nerr:.1e}, zeros {np.mean(z == 0):.2f}")
            assert err <= TOL, (name, k, t, err)
            assert nerr <= 1e-12
            assert np.all(z >= 0)
            x_in = z
            xp = y


def test_gnn_identity_weight_is_relu_of_the_product():
    """With W = I every matrix-core sum adds exact zeros to one product, so the
    output is ReLU of the plain product to the bit (up to the sign of zero)."""
    M = W.make_matrix("rmat", 12, "row_normalized", 75, 76, 16)
    d = A_.Decomposition.from_matrix(M, 64, seed=4)
    plan = A_.Plan(d)
    for k in (32, 64):
        X = W.features(M.n, k, 950 + k)
        xp = plan.empty(k)
        plan.permute_in(torch.from_numpy(X).cuda(), xp)
        ws = plan.workspace(plan.workspace_size(k))
        y0, y1 = plan.empty(k), plan.empty(k)
        plan.spmm([A_.operand(xp, y0)], ws)
        eye = torch.eye(k, dtype=torch.float32, device="cuda")
        plan.spmm([A_.operand(xp, y1, w=eye)], ws)
        torch.cuda.synchronize()
        assert torch.equal(torch.clamp(y0, min=0.0), y1)


def test_gnn_operand_alone_equals_in_a_mix():
    M = W.make_matrix("grid3d", 16, "sym_laplacian", 77, 78)
    d = A_.Decomposition.from_matrix(M, 256, seed=6)
    plan = A_.Plan(d)
    k = 32
    Wm = torch.randn((k, k), generator=torch.Generator().manual_seed(5)).cuda() / k ** 0.5
    xs = []
    for i in range(3):
        xp = plan.empty(k)
        plan.permute_in(torch.from_numpy(W.features(M.n, k, 960 + i)).cuda(), xp)
        xs.append(xp)
    ws1 = plan.workspace(plan.workspace_size(k))
    alone = []
    for i, xp in enumerate(xs):
        y = plan.empty(k)
        plan.spmm([A_.operand(xp, y, w=Wm if i != 1 else None)], ws1)
        alone.append(y)
    ys = [plan.empty(k) for _ in xs]
    ops = [A_.operand(xp, y, w=Wm if i != 1 else None) for i, (xp, y) in enumerate(zip(xs, ys))]
    plan.spmm(ops, plan.workspace(3 * plan.workspace_size(k)))
    ys_static = [plan.empty(k) for _ in xs]
    plan.spmm_static([A_.operand(xp, y, w=Wm if i != 1 else None)
                      for i, (xp, y) in enumerate(zip(xs, ys_static))])
    torch.cuda.synchronize()
    for a, b_, c in zip(alone, ys, ys_static):
        assert torch.equal(a, b_) and torch.equal(a, c)


def test_gnn_rejects_unsupported_operands():
    M = W.make_matrix("grid2d", 16, "uniform", 79, 80)
    plan = A_.Plan(A_.Decomposition.from_matrix(M, 16, seed=1))
    ws = plan.workspace(plan.workspace_size(64, "bf16") + plan.workspace_size(48))
    w64 = torch.eye(64, device="cuda")
    with pytest.raises(A_.ArrowError) as e:
        plan.spmm([A_.operand(plan.empty(64, "bf16"), plan.empty(64, "bf16"), "bf16",
                              w=w64)], ws)
    assert e.value.status == A_.ERR_UNSUPPORTED
    w48 = torch.eye(48, device="cuda")
    with pytest.raises(A_.ArrowError) as e:
        plan.spmm([A_.operand(plan.empty(48), plan.empty(48), w=w48)], ws)
    assert e.value.status == A_.ERR_UNSUPPORTED
