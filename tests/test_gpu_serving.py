"""Serving form on the GPU: requests on different graphs, widths and dtypes
arrive as a Poisson stream, are admitted by HBM footprint and batched per
(graph, dtype); each result is the same alone and in the mix (bitwise: the
per-request arithmetic does not depend on the other requests), and matches the
FP64 oracle within the dtype's tolerance."""
import numpy as np
import pytest

import workloads as W
from oracle import spmm as S
from tests.gpu_helpers import say

torch = pytest.importorskip("torch")
A_ = pytest.importorskip("paper_2402_19364_amd")
from paper_2402_19364_amd.serve import GpuEngine, Request, Server, latency_stats  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _pool():
    mats = {
        "grid3d_16": (W.make_matrix("grid3d", 16, "sym_laplacian", 0, 0), 256),
        "grid3d_24": (W.make_matrix("grid3d", 24, "sym_laplacian", 0, 0), 576),
        "rmat_12": (W.make_matrix("rmat", 12, "row_normalized", 5, 6, 8), 128),
        "rmat_13": (W.make_matrix("rmat", 13, "row_normalized", 7, 8, 16), 256),
    }
    decs = {name: A_.Decomposition.from_matrix(M, b, seed=1) for name, (M, b) in mats.items()}
    return mats, decs


def _requests(mats, count, rate, seed):
    rng = np.random.default_rng(seed)
    names = sorted(mats)
    t = 0.0
    reqs = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        g = names[rng.integers(len(names))]
        k = int(rng.choice([16, 32, 64, 128]))
        dtype = "f32" if rng.random() < 0.6 else "bf16"
        reqs.append(Request(rid, g, None, int(rng.integers(3, 9)), dtype, t, width=k,
                            x0_seed=10_000 + rid))
    return reqs


def _clone(r: Request) -> Request:
    return Request(r.rid, r.graph, None, r.iters, r.dtype, 0.0, width=r.width,
                   x0_seed=r.x0_seed)


def test_alone_equals_mix_and_oracle():
    mats, decs = _pool()
    reqs = _requests(mats, 24, rate=2000.0, seed=3)
    say(f"[serving] {len(reqs)} requests over {len(mats)} graphs")
    srv = Server(GpuEngine(0), hbm_budget=2 << 30)
    for name, d in decs.items():
        srv.register_graph(name, d)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    # the admission estimate of every plan bounds its actual device bytes
    for name, (handle, fp) in srv.plans.items():
        est = srv.engine.plan_footprint(decs[name])
        say(f"[serving] plan {name}: {fp} bytes, admission estimate {est}")
        assert fp == handle.footprint() <= est
    assert srv.max_group_width >= 2, "no batching happened"
    stats = latency_stats(done)
    say(f"[serving] mix: p50 {stats['p50_ms']:.2f} ms p99 {stats['p99_ms']:.2f} ms, "
        f"widest batch {srv.max_group_width}, peak {srv.peak_used / 2**20:.1f} MiB")
    for r in reqs:
        alone = _clone(r)
        srv1 = Server(GpuEngine(0), hbm_budget=2 << 30)
        srv1.register_graph(r.graph, decs[r.graph])
        srv1.run([alone])
        assert np.array_equal(alone.result, r.result), r.rid
        assert np.array_equal(alone.norms, r.norms), r.rid
    # oracle: FP32 requests against the FP64 trajectory (X_T normalised), BF16 within its
    # per-step bound compounded over T steps
    for r in reqs[:8]:
        M = mats[r.graph][0]
        gen = torch.Generator(device="cuda")
        gen.manual_seed(r.x0_seed)
        x0 = torch.randn((M.n, r.k), generator=gen, dtype=torch.float32, device="cuda")
        X0 = x0.cpu().numpy().astype(np.float64)
        if r.dtype == "bf16":
            from oracle import quant as Q
            X0 = Q.quantize(X0, "bf16")
        Ys, nus = S.iterate(M, X0, r.iters)
        ref = Ys[-1] / nus[-1][None, :]
        tol = 1e-5 if r.dtype == "f32" else 4e-3 * r.iters
        err = S.rel_fro(r.result, ref)
        say(f"[serving] request {r.rid} {r.graph} k={r.k} {r.dtype} T={r.iters}: err {err:.2e}")
        assert err <= tol, (r.rid, err)
