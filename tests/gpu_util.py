"""Helpers shared by the GPU tests: run the library through the C ABI and
compare with the FP64 oracle."""

from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2503_18198_amd import capi


def dev_factors(factors, dtype=torch.float32):
    return [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to("cuda").to(dtype).contiguous()
            for f in factors]


def gpu_mttkrp(h, mode, dfac, R, bf16=False):
    out = torch.full((h.dims[mode], R), float("nan"), dtype=torch.float32, device="cuda")
    fac = [None if m == mode else dfac[m] for m in range(len(dfac))]
    if bf16:
        capi.mttkrp_run_bf16(h, mode, fac, out, R)
    else:
        capi.mttkrp_run(h, mode, fac, out, R)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def rel_fro(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def oracle_mttkrp(t_idx, t_val, dims, factors, mode, threads=8):
    return oracle.mttkrp(t_idx, t_val.astype(np.float64), dims, [np.asarray(f, dtype=np.float64) for f in factors],
                         mode, threads=threads)
