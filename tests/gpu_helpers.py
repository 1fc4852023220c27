"""Shared helpers of the GPU tests (not collected by pytest)."""
from __future__ import annotations

import sys

import numpy as np

import paper_2402_19364_amd as A_


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def to_device_csr(M, torch):
    rp = torch.from_numpy(M.row_ptr.astype(np.int32)).cuda()
    col = torch.from_numpy(M.col.astype(np.int32)).cuda()
    val = torch.from_numpy(M.val.astype(np.float32)).cuda()
    return rp, col, val


def plan_order_to_orig(y_plan: np.ndarray, vop0: np.ndarray) -> np.ndarray:
    out = np.empty_like(y_plan)
    out[vop0] = y_plan
    return out


def run_steps(plan, x_plan, T, torch, dtype="f32", renorm=True, x_scale=None):
    """T products chained through arrow_spmm (the operand API), keeping every
    stored Y_t.  Returns (ys, norms, scales): device tensors per step."""
    k = x_plan.shape[1]
    ws = plan.workspace(plan.workspace_size(k, dtype))
    dev = x_plan.device
    inv = [torch.zeros(k, dtype=torch.float64, device=dev) for _ in range(2)]
    mx = [torch.zeros(k, dtype=torch.float32, device=dev) for _ in range(2)]
    ys, norms, scales = [], [], []
    cur, cur_scale = x_plan, x_scale
    for t in range(T):
        y = plan.empty(k, dtype)
        nrm = torch.zeros(k, dtype=torch.float64, device=dev)
        ysc = torch.ones(k, dtype=torch.float32, device=dev)
        scaled = dtype in ("f16", "f8e4m3")
        op = A_.operand(cur, y, dtype,
                        x_scale=cur_scale,
                        x_inv_norm=inv[(t - 1) % 2] if (t > 0 and renorm) else None,
                        x_maxabs=mx[(t - 1) % 2] if (t > 0 and scaled) else None,
                        y_scale=ysc if scaled else None,
                        y_maxabs=mx[t % 2] if scaled else None,
                        y_norm=nrm, y_inv_norm=inv[t % 2])
        plan.spmm([op], ws)
        ys.append(y)
        norms.append(nrm)
        scales.append(ysc)
        cur, cur_scale = y, (ysc if scaled else None)
    torch.cuda.synchronize()
    return ys, norms, scales


def stored_values(y, dtype, torch) -> np.ndarray:
    """Stored plan-order values as float64 (codes decoded with the oracle's
    format definitions for the reduced types)."""
    from oracle import quant as Q
    if dtype == "f32":
        return y.cpu().numpy().astype(np.float64)
    if dtype in ("bf16", "f16"):
        codes = y.view(torch.int16).cpu().numpy().view(np.uint16)
        return Q.decode(codes, dtype)
    codes = y.view(torch.uint8).cpu().numpy()
    return Q.decode(codes, "f8e4m3")
