"""GPU parity of the FP32 iterated arrow SpMM against the FP64 oracle.

Gate (per iteration, relative Frobenius error over the n x k result):
free-running -- the GPU trajectory from the seeded X_0 against the oracle's own
FP64 trajectory from the same X_0 -- within 1e-5.  The teacher-forced error (one
oracle step from exactly the X_t the GPU consumed) is checked too; it isolates
the error of a single product.
"""
import numpy as np
import pytest

import workloads as W
from oracle import decomp as D
from oracle import spmm as S
from tests.gpu_helpers import plan_order_to_orig, run_steps, say, to_device_csr

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


def _check_trajectory(M, b, k, T, seed_x=7, la=0, decomp_seed=1, ld=None, label=""):
    say(f"[parity] {label} n={M.n} nnz={M.nnz} b={b} k={k} T={T} la={la} ld={ld}")
    d = A_.Decomposition.from_matrix(M, b, seed=decomp_seed, la=la)
    levels = d.levels()
    D.validate(M, levels, b)
    vop0 = levels[0]["vop"].astype(np.int64)
    plan = A_.Plan(d)
    assert plan.footprint() == plan.info()["footprint_bytes"] > 0 or M.nnz == 0
    X0 = W.features(M.n, k, seed_x)
    ldx = ld or k
    xs = torch.zeros((M.n, ldx), dtype=torch.float32, device="cuda")
    xs[:, :k] = torch.from_numpy(X0).cuda()
    x_orig = xs[:, :k]
    xp_full = torch.zeros((M.n, ldx), dtype=torch.float32, device="cuda")
    x_plan = xp_full[:, :k]
    plan.permute_in(x_orig, x_plan)
    torch.cuda.synchronize()
    assert np.array_equal(x_plan.cpu().numpy(), X0[vop0])
    ys, norms, _ = run_steps(plan, x_plan, T, torch)
    ref_Y, ref_nu = S.iterate(M, X0.astype(np.float64), T)
    prev = None
    worst_tf = worst_fr = 0.0
    for t in range(T):
        y = plan_order_to_orig(ys[t].cpu().numpy().astype(np.float64), vop0)
        nu = norms[t].cpu().numpy()
        # free running against the oracle's own trajectory
        fr = S.rel_fro(y, ref_Y[t])
        assert fr <= TOL, (t, fr)
        assert np.allclose(nu, ref_nu[t], rtol=TOL, atol=0), t
        # norms of the stored result, exactly as FP64 sums of the stored values
        assert np.allclose(nu, np.sqrt(S.col_sumsq(y)), rtol=1e-12, atol=0)
        # teacher forced: one oracle step from the GPU's own input
        x_in = X0.astype(np.float64) if t == 0 else prev / np.where(
            pnu > 0, pnu, 1.0)[None, :] * (pnu > 0)[None, :]
        tf = S.rel_fro(y, S.csr_spmm(M, x_in))
        assert tf <= TOL, (t, tf)
        worst_tf, worst_fr = max(worst_tf, tf), max(worst_fr, fr)
        prev, pnu = y, nu
    say(f"[parity] {label} ok: worst teacher-forced {worst_tf:.2e} free-running {worst_fr:.2e}")
    # arrow_spmm_iterate runs the same kernels: bitwise equal final product
    y_it = torch.zeros((M.n, ldx), dtype=torch.float32, device="cuda")[:, :k]
    nrm = torch.zeros(T * k, dtype=torch.float64, device="cuda")
    plan.iterate(x_plan, y_it, T, norms=nrm)
    torch.cuda.synchronize()
    assert torch.equal(y_it, ys[-1])
    for T2 in (1, 2):  # both parities of the ping-pong through the compact scratch buffer
        y2 = torch.zeros((M.n, ldx), dtype=torch.float32, device="cuda")[:, :k]
        plan.iterate(x_plan, y2, T2)
        torch.cuda.synchronize()
        assert torch.equal(y2, ys[T2 - 1]), T2
    assert torch.equal(nrm.view(T, k), torch.stack(norms))
    # permute_out with the last normalisation gives X_T in the original order
    out = torch.empty((M.n, k), dtype=torch.float32, device="cuda")
    inv = torch.where(norms[-1] > 0, 1.0 / norms[-1], torch.zeros_like(norms[-1]))
    plan.permute_out(ys[-1], out, col_factor=inv)
    torch.cuda.synchronize()
    expect = plan_order_to_orig(ys[-1].cpu().numpy().astype(np.float64), vop0) * \
        inv.cpu().numpy()[None, :]
    assert np.allclose(out.cpu().numpy(), expect, rtol=1e-6, atol=1e-30)
    return plan


def test_config_grid64_full():
    w = W.WORKLOADS["grid64"]
    M = W.workload_matrix(w)
    _check_trajectory(M, w.b, w.k, w.iters, seed_x=w.seeds["x"],
                      decomp_seed=w.seeds["decompose"], label="grid64 random-forest")
    _check_trajectory(M, w.b, w.k, w.iters, seed_x=w.seeds["x"], la=A_.LA_IDENTITY,
                      label="grid64 identity")


@pytest.mark.parametrize("k", [16, 32, 48, 64, 128, 144])
def test_rmat_multilevel_widths(k):
    M = W.make_matrix("rmat", 13, "row_normalized", 31, 32, 16)
    _check_trajectory(M, 64, k, 4, seed_x=k, label=f"rmat13 k={k}")


def test_strided_rows_and_hubs():
    # hubs: a star over everything plus a random graph -> long rows at every level
    n = 6000
    rng = np.random.default_rng(3)
    edges = [(0, i) for i in range(1, n)] + [(1, i) for i in range(2, n, 3)]
    edges += [(int(a), int(b)) for a, b in rng.integers(0, n, (20000, 2)) if a != b]
    M = W.from_edges(n, edges, values="uniform", seed=5, diagonal=True)
    _check_trajectory(M, 16, 32, 3, ld=48, label="hubs ld=48")


@pytest.mark.parametrize("k", [16, 32, 64, 128])
def test_long_partial_row_lists_are_combined(k):
    # a hub row cut into about 150 chunks lists all of their partial rows:
    # the combine pass sums them before the level-0 pass (every tile width of
    # its kernel; the scaled formats meet it in the full-size R-MAT tests)
    n = 10000
    rng = np.random.default_rng(8)
    edges = [(0, i) for i in range(1, n)]
    edges += [(int(a), int(b)) for a, b in rng.integers(0, n, (30000, 2)) if a != b]
    M = W.from_edges(n, edges, values="uniform", seed=9, diagonal=True)
    plan = _check_trajectory(M, 16, k, 3, label=f"combined lists k={k}")
    assert plan.kernel_bytes(A_.KERNEL_COMBINE, k) > 0
    plan.profile(True)
    x = plan.empty(k)
    x.copy_(torch.from_numpy(W.features(M.n, k, 1)).cuda())
    run_steps(plan, x, 1, torch)
    torch.cuda.synchronize()
    assert plan.profile_query(A_.KERNEL_COMBINE)[0] >= 1
    plan.profile(False)


def test_gather_batches_agree():
    # rows longer than every short batch and rows listing more than 2 partial
    # rows: each batch must give the same products (the schedule changes, the
    # summation order does not); the FP64 norms sum the same squares in
    # another fixed order, so they agree to rounding
    M = W.make_matrix("rmat", 12, "row_normalized", 51, 52, 16)
    d = A_.Decomposition.from_matrix(M, 32, seed=2)
    plan = A_.Plan(d)
    inf = plan.info()
    assert inf["level0_batch"] == 0 and inf["levels"] > 2
    vop0 = d.level(0)["vop"].astype(np.int64)
    X0 = W.features(M.n, 32, 4)
    x = plan.empty(32)
    plan.permute_in(torch.from_numpy(X0).cuda(), x)
    base, base_nu, _ = run_steps(plan, x, 2, torch)
    ref = S.csr_spmm(M, X0.astype(np.float64))
    for batch in (4, 5, 6, 7, 8, -1):
        say(f"[parity] rmat12 gather batch {batch}")
        plan.set_batch(A_.KERNEL_UPPER, batch)
        plan.set_batch(A_.KERNEL_LEVEL0, batch)
        ys, nus, _ = run_steps(plan, x, 2, torch)
        for t in range(2):
            assert torch.equal(ys[t], base[t]), (batch, t)
            assert torch.allclose(nus[t], base_nu[t], rtol=1e-13, atol=0), (batch, t)
        y0 = plan_order_to_orig(ys[0].cpu().numpy().astype(np.float64), vop0)
        assert S.rel_fro(y0, ref) <= TOL
    assert plan.info()["level0_batch"] == inf["level0_batch"]
    with pytest.raises(A_.ArrowError):
        plan.set_batch(A_.KERNEL_LEVEL0, 9)
    with pytest.raises(A_.ArrowError):
        plan.set_batch(A_.KERNEL_NORM, 5)


def test_short_batch_chosen_for_stencils():
    # identity arrangement with the whole stencil inside the band: one level
    for shape, size, b, expect in (("grid2d", 24, 40, 5), ("grid3d", 10, 100, 7)):
        M = W.make_matrix(shape, size, "sym_laplacian", 0, 0)
        plan = A_.Plan(A_.Decomposition.from_matrix(M, b, seed=1, la=A_.LA_IDENTITY))
        assert plan.info()["level0_batch"] == expect, shape
        _check_trajectory(M, b, 16, 2, la=A_.LA_IDENTITY, label=f"{shape} short batch")


def test_separator_arrangement_products():
    """The product over decompositions built with the separator arrangement
    (Section 5.2): more levels than the forest on grids, folded and listed
    rows alike."""
    for M, b in ((W.make_matrix("grid2d", 48, "sym_laplacian", 81, 82), 48),
                 (W.make_matrix("grid3d", 14, "sym_laplacian", 83, 84), 196),
                 (W.make_matrix("rmat", 12, "row_normalized", 85, 86, 16), 64)):
        _check_trajectory(M, b, 32, 4, la=A_.LA_SEPARATOR, label="separator arrangement")


def test_wide_arrow_int32_codes():
    # b > 21845 switches the level-0 pass to 32-bit columns
    M = W.make_matrix("grid2d", 190, "sym_laplacian", 0, 0)
    _check_trajectory(M, 22000, 16, 3, label="grid190 b=22000")


def test_degenerate_inputs():
    for label, M, b in (
        ("empty", W.from_edges(300, []), 4),
        ("diagonal", W.from_edges(257, [], diagonal=True, values="uniform"), 4),
        ("n<b", W.random_graph(50, 0.2, 2, diagonal=True), 64),
        ("single", W.from_edges(1, [], diagonal=True, values="uniform"), 2),
        ("ragged", W.make_matrix("grid2d", 37, "uniform", 3, 4), 5),
    ):
        _check_trajectory(M, b, 16, 2, label=label)


def test_plain_csr_baseline():
    M = W.make_matrix("rmat", 12, "row_normalized", 1, 2, 16)
    rp, col, val = to_device_csr(M, torch)
    X = W.features(M.n, 64, 9)
    x = torch.from_numpy(X).cuda()
    y = torch.empty_like(x)
    ws = torch.empty(A_.csr_workspace_size(M.n, 64), dtype=torch.uint8, device="cuda")
    nrm = torch.empty(64, dtype=torch.float64, device="cuda")
    ref = S.csr_spmm(M, X)
    first = None
    for batch in (A_.csr_batch(M.row_ptr), 4, 5, 8):
        A_.csr_spmm(M.n, rp, col, val, x, y, sumsq_ws=ws.view(torch.float64), norms=nrm,
                    batch=batch)
        torch.cuda.synchronize()
        assert S.rel_fro(y.cpu().numpy(), ref) <= TOL
        assert np.allclose(nrm.cpu().numpy(), np.linalg.norm(ref, axis=0), rtol=TOL)
        if first is None:
            first = y.clone()
        assert torch.equal(y, first), batch
    with pytest.raises(A_.ArrowError):
        A_.csr_spmm(M.n, rp, col, val, x, y, batch=3)


def test_copy_kernel():
    a = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    A_.copy(a, b, a.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_argument_errors_on_device():
    M = W.make_matrix("grid2d", 16, "uniform", 0, 1)
    d = A_.Decomposition.from_matrix(M, 8)
    plan = A_.Plan(d)
    x = plan.empty(16)
    y = plan.empty(16)
    ws = plan.workspace(plan.workspace_size(16))
    with pytest.raises(A_.ArrowError):           # aliasing
        plan.spmm([A_.operand(x, x)], ws)
    with pytest.raises(A_.ArrowError):           # k not a multiple of 16
        plan.spmm([A_.operand(x[:, :8], y[:, :8])], ws)
    with pytest.raises(A_.ArrowError):           # workspace too small
        plan.spmm([A_.operand(x, y)], ws[:128])
    with pytest.raises(A_.ArrowError):           # F8 without y_scale
        plan.spmm([A_.operand(plan.empty(16, "f8e4m3"), plan.empty(16, "f8e4m3"), "f8e4m3")],
                  plan.workspace(plan.workspace_size(16, "f8e4m3")))
    info = plan.info()
    assert info["n"] == M.n and info["levels"] >= 1
