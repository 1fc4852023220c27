"""Precision form on the GPU: X/Y stored BF16, FP16 or FP8-E4M3 with per-column
power-of-two scales, FP32 accumulation, FP64 column norms.

Gate, per step (teacher forced: one oracle product from exactly the stored
X_t the GPU consumed, decoded with the oracle's own format definitions):

* every stored element within one storage quantum of the FP64 product (round
  to nearest of an FP32 accumulator that is itself within ~1e-6 relative),
* relative Frobenius error within the rounding bound u = 2^-(p+1) plus margin:
  FP16 5e-4, BF16 4e-3, FP8 6.3e-2,
* the scale is a power of two and no stored value overflowed,
* the FP64 norms equal the norms of the stored values.
The 50-iteration drift against the oracle's own FP64 trajectory is reported.
"""
import numpy as np
import pytest

import workloads as W
from oracle import quant as Q
from oracle import spmm as S
from tests.gpu_helpers import plan_order_to_orig, run_steps, say, stored_values

torch = pytest.importorskip("torch")
A_ = pytest.importorskip("paper_2402_19364_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _decoded(y, dtype, scale):
    v = stored_values(y, dtype, torch)
    if scale is not None:
        v = v * scale.cpu().numpy().astype(np.float64)[None, :]
    return v


def _check(M, b, k, T, dtype, label, drift_T=0):
    say(f"[precision] {label} dtype={dtype} n={M.n} nnz={M.nnz} k={k} T={T}")
    d = A_.Decomposition.from_matrix(M, b, seed=3)
    vop0 = d.level(0)["vop"].astype(np.int64)
    plan = A_.Plan(d)
    X0 = W.features(M.n, k, 11)
    x = torch.from_numpy(X0).cuda()
    xp = plan.empty(k, dtype)
    scaled = dtype in ("f16", "f8e4m3")
    xs = torch.zeros(k, dtype=torch.float32, device="cuda") if scaled else None
    xm = torch.zeros(k, dtype=torch.float32, device="cuda") if scaled else None
    plan.permute_in(x, xp, dtype, x_scale=xs, x_maxabs=xm)
    torch.cuda.synchronize()
    # quantised input: nearest representable value of X0 / scale
    x_dec = plan_order_to_orig(_decoded(xp, dtype, xs), vop0)
    if scaled:
        s = xs.cpu().numpy().astype(np.float64)
        assert np.all(np.exp2(np.round(np.log2(s))) == s)
        assert np.all(np.max(np.abs(X0), axis=0) / s <= Q.FORMATS[dtype][2])
        expect = Q.quantize(X0.astype(np.float64) / s[None, :], dtype) * s[None, :]
        codes_max = np.max(np.abs(stored_values(xp, dtype, torch)), axis=0)
        assert np.array_equal(xm.cpu().numpy().astype(np.float64), codes_max)
    elif dtype == "f32":
        expect = X0.astype(np.float64)
    else:
        expect = Q.quantize(X0.astype(np.float64), dtype)
    assert np.array_equal(x_dec, expect)

    steps = max(T, drift_T)
    ys, norms, scales = run_steps(plan, xp, steps, torch, dtype=dtype, x_scale=xs)
    bound = Q.STEP_BOUND[dtype]
    x_in = x_dec
    worst = 0.0
    for t in range(T):
        sc = scales[t] if scaled else None
        y = plan_order_to_orig(_decoded(ys[t], dtype, sc), vop0)
        ref = S.csr_spmm(M, x_in)
        err = S.rel_fro(y, ref)
        worst = max(worst, err)
        assert err <= bound, (t, err)
        if scaled:
            c = sc.cpu().numpy().astype(np.float64)
            assert np.all(np.exp2(np.round(np.log2(c))) == c)
            assert np.all(np.max(np.abs(ref), axis=0) / c <= Q.FORMATS[dtype][2] * (1 + 1e-6))
        else:
            c = np.ones(k)
        if dtype != "f32":
            # rounding to the stored format (one quantum covers a boundary flip)
            # plus the FP32 accumulation error, bounded by ~m 2^-24 (|A| |x|)
            quantum = Q.spacing(ref / c[None, :], dtype) * c[None, :]
            Aabs = W.CSR(M.n, M.row_ptr, M.col, np.abs(M.val))
            slack = 1e-5 * S.csr_spmm(Aabs, np.abs(x_in)) + 1e-30
            assert np.all(np.abs(y - ref) <= quantum + slack), t
        nu = norms[t].cpu().numpy()
        assert np.allclose(nu, np.sqrt(S.col_sumsq(y)), rtol=1e-12, atol=0)
        inv = np.where(nu > 0, 1.0 / np.where(nu > 0, nu, 1.0), 0.0)
        x_in = y * inv[None, :]
    say(f"[precision] {label} {dtype}: worst per-step error {worst:.3e} (bound {bound:g})")
    if drift_T:
        ref_Y, _ = S.iterate(M, X0.astype(np.float64), drift_T)
        sc = scales[drift_T - 1] if scaled else None
        y = plan_order_to_orig(_decoded(ys[drift_T - 1], dtype, sc), vop0)
        drift = S.rel_fro(y / np.linalg.norm(y, axis=0),
                          ref_Y[-1] / np.linalg.norm(ref_Y[-1], axis=0))
        say(f"[precision] {label} {dtype}: drift after {drift_T} iterations {drift:.3e} "
            f"(reported, not gated)")


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f8e4m3"])
def test_grid3d_precision(dtype):
    M = W.make_matrix("grid3d", 20, "sym_laplacian", 0, 0)
    _check(M, 400, 128, 4, dtype, "grid3d 20^3", drift_T=50)


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f8e4m3"])
def test_rmat_precision(dtype):
    M = W.make_matrix("rmat", 13, "row_normalized", 41, 42, 16)
    _check(M, 64, 32, 4, dtype, "rmat13", drift_T=50)


def test_f32_scales_are_ignored():
    M = W.make_matrix("grid2d", 20, "uniform", 0, 1)
    _check(M, 8, 16, 2, "f32", "grid20")
