"""GPU parity at the benchmark's full sizes, in the launch sequence bench.py
times: permute_in, T chained products over all k columns through arrow_spmm
(1/nu of step t-1 folded into step t, two ping-pong buffers), permute_out with
the last 1/nu.  The oracle follows sampled columns only: the iteration is
column-separable (each column is normalised on its own), so the FP64 CSR
iteration of a few columns of X_0 at full n is the exact reference for them.

Gates: FP32 -- X_T and every nu_t within 1e-5 (relative) on the sampled
columns.  BF16 / FP8 -- the first product, teacher-forced from the stored
X_0, within the per-step bound on the sampled columns; the drift of X_T after
T steps against the FP64 trajectory is reported.
"""
import time

import numpy as np
import pytest

import workloads as W
from oracle import quant as Q
from oracle import spmm as S
from tests.gpu_helpers import say

torch = pytest.importorskip("torch")
A_ = pytest.importorskip("paper_2402_19364_amd")

pytestmark = pytest.mark.gpu

TOL = 1e-5
_CACHE = {}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    _CACHE.clear()


def _plan(name):
    """Matrix, decomposition and plan of a workload (cached per module)."""
    if name not in _CACHE:
        w = W.WORKLOADS[name]
        t0 = time.perf_counter()
        M = W.workload_matrix(w)
        say(f"[full] {name}: n={M.n} nnz={M.nnz} generated in {time.perf_counter() - t0:.1f}s")
        t0 = time.perf_counter()
        d = A_.Decomposition.from_matrix(M, w.b, seed=w.seeds["decompose"])
        plan = A_.Plan(d)
        vop0 = d.level(0)["vop"].astype(np.int64)
        say(f"[full] {name}: {d.info()['levels']} levels, plan in {time.perf_counter() - t0:.1f}s")
        _CACHE.clear()  # one full-size plan resident at a time
        _CACHE[name] = (w, M, plan, vop0)
    return _CACHE[name]


def _sample_cols(k):
    return sorted({0, k // 3, (2 * k) // 3, k - 1})


def _run(plan, X0, dtype, T, cols):
    """bench.py's launch sequence; returns the sampled columns of X_T (FP32,
    original order), the per-step norms [T, k] and the stored first product
    with its scale."""
    n, k = X0.shape
    dev = "cuda"
    scaled = dtype in ("f16", "f8e4m3")
    x = torch.from_numpy(X0).to(dev)
    xp = plan.empty(k, dtype)
    xs = torch.ones(k, dtype=torch.float32, device=dev)
    xm = torch.zeros(k, dtype=torch.float32, device=dev)
    plan.permute_in(x, xp, dtype, x_scale=xs if scaled else None, x_maxabs=xm if scaled else None)
    bufs = [plan.empty(k, dtype), plan.empty(k, dtype)]
    inv = [torch.zeros(k, dtype=torch.float64, device=dev) for _ in range(2)]
    scl = [torch.ones(k, dtype=torch.float32, device=dev) for _ in range(2)]
    mx = [torch.zeros(k, dtype=torch.float32, device=dev) for _ in range(2)]
    norms = torch.zeros((T, k), dtype=torch.float64, device=dev)
    ws = plan.workspace(plan.workspace_size(k, dtype))
    cur, cur_s, cur_m = xp, (xs if scaled else None), (xm if scaled else None)
    first = None
    for t in range(T):
        y = bufs[t % 2]
        op = A_.operand(cur, y, dtype, x_scale=cur_s,
                        x_inv_norm=inv[(t - 1) % 2] if t > 0 else None,
                        x_maxabs=cur_m,
                        y_scale=scl[t % 2] if scaled else None,
                        y_maxabs=mx[t % 2] if scaled else None,
                        y_norm=norms[t], y_inv_norm=inv[t % 2])
        plan.spmm([op], ws)
        if t == 0:
            torch.cuda.synchronize()
            first = (y.clone(), scl[0].clone() if scaled else None)
        cur, cur_s, cur_m = y, (scl[t % 2] if scaled else None), (mx[t % 2] if scaled else None)
    out = torch.empty((n, k), dtype=torch.float32, device=dev)
    plan.permute_out(cur, out, dtype, x_scale=cur_s, col_factor=inv[(T - 1) % 2])
    torch.cuda.synchronize()
    xs_host = xs.cpu().numpy().astype(np.float64) if scaled else None
    xt = out[:, cols].cpu().numpy().astype(np.float64)
    return xt, norms.cpu().numpy(), first, xp, xs_host


def _oracle(M, X0c, T):
    """FP64 trajectory of the sampled columns: X_T and the norms of every step."""
    X = X0c.astype(np.float64)
    nus = []
    for _ in range(T):
        nu, X = S.renormalize(S.csr_spmm(M, X))
        nus.append(nu)
    return X, np.array(nus)


def _decoded_plan_to_orig(y, dtype, scale, vop0, cols):
    """Stored plan-order values of the sampled columns, decoded (oracle format
    definitions), in the original order."""
    if dtype == "f32":
        v = y[:, cols].cpu().numpy().astype(np.float64)
    elif dtype in ("bf16", "f16"):
        v = Q.decode(y.view(torch.int16)[:, cols].cpu().numpy().view(np.uint16), dtype)
    else:
        v = Q.decode(y.view(torch.uint8)[:, cols].cpu().numpy(), "f8e4m3")
    if scale is not None:
        v = v * np.asarray(scale, np.float64)[cols][None, :]
    out = np.empty_like(v)
    out[vop0] = v
    return out


@pytest.mark.parametrize("name", ["grid2048", "rmat22"])
def test_full_size_fp32(name):
    w, M, plan, vop0 = _plan(name)
    X0 = W.features(M.n, w.k, w.seeds["x"])
    cols = _sample_cols(w.k)
    XT, norms, _, _, _ = _run(plan, X0, "f32", w.iters, cols)
    t0 = time.perf_counter()
    ref_X, ref_nu = _oracle(M, X0[:, cols], w.iters)
    err = S.rel_fro(XT, ref_X)
    nerr = float(np.max(np.abs(norms[:, cols] - ref_nu) / ref_nu))
    say(f"[full] {name} f32 k={w.k} T={w.iters}: X_T error {err:.2e}, worst norm error "
        f"{nerr:.2e} on columns {cols} (oracle {time.perf_counter() - t0:.1f}s)")
    assert err <= TOL
    assert nerr <= TOL


@pytest.mark.parametrize("name,dtype", [("grid3d160", "bf16"), ("grid3d160", "f8e4m3"),
                                        ("rmat22_k128", "bf16"), ("rmat22_k128", "f8e4m3")])
def test_full_size_precision(name, dtype):
    w, M, plan, vop0 = _plan(name)
    X0 = W.features(M.n, w.k, w.seeds["x"])
    cols = _sample_cols(w.k)
    XT, norms, (y0, s0), xp, xs = _run(plan, X0, dtype, w.iters, cols)
    # first product, teacher forced from the stored X_0 of the sampled columns
    x0_dec = _decoded_plan_to_orig(xp, dtype, xs, vop0, cols)
    y0_dec = _decoded_plan_to_orig(y0, dtype, None if s0 is None else s0.cpu().numpy(), vop0,
                                   cols)
    ref0 = S.csr_spmm(M, x0_dec)
    step = S.rel_fro(y0_dec, ref0)
    # drift of the free-running trajectory after T steps
    ref_X, _ = _oracle(M, X0[:, cols], w.iters)
    drift = S.rel_fro(XT, ref_X)
    say(f"[full] {name} {dtype} k={w.k} T={w.iters}: first-step error {step:.2e} "
        f"(bound {Q.STEP_BOUND[dtype]:g}), drift after {w.iters} steps {drift:.2e} "
        f"(reported) on columns {cols}")
    assert step <= Q.STEP_BOUND[dtype]
    assert np.all(np.isfinite(XT)) and np.all(norms[:, cols] > 0)
