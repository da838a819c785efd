"""Upload seeded Darcy systems to device memory (PyTorch tensors) as libskr operators.

Input marshalling only: no arithmetic of the method happens here.
"""
from __future__ import annotations

import numpy as np


def upload_systems(systems, device="cuda:0", kind="csr"):
    """Return (ops, b_list, x_list) for ``systems`` (list of DarcySystem) on ``device``.

    kind = "csr" (CSR matrices) or "stencil" (matrix-free face coefficients: 5-point for 2-D systems,
    7-point for 3-D ones). The x tensors are zero-initialised outputs.
    """
    import torch
    from paper_2401_09516_amd.skr import csr_op, stencil7_op, stencil_op

    ops, bs, xs = [], [], []
    for s in systems:
        n = s.n
        if kind == "csr":
            rp = torch.from_numpy(np.ascontiguousarray(s.A.indptr, dtype=np.int32)).to(device)
            ci = torch.from_numpy(np.ascontiguousarray(s.A.indices, dtype=np.int32)).to(device)
            va = torch.from_numpy(np.ascontiguousarray(s.A.data, dtype=np.float64)).to(device)
            ops.append(csr_op(rp, ci, va, n))
        elif kind == "stencil":
            ax = torch.from_numpy(np.ascontiguousarray(s.ax, dtype=np.float64).ravel()).to(device)
            ay = torch.from_numpy(np.ascontiguousarray(s.ay, dtype=np.float64).ravel()).to(device)
            if hasattr(s, "az"):
                az = torch.from_numpy(np.ascontiguousarray(s.az, dtype=np.float64).ravel()).to(device)
                ops.append(stencil7_op(ax, ay, az, s.N, s.N, s.N, s.inv_h2))
            else:
                ops.append(stencil_op(ax, ay, s.N_g, s.N_g, s.inv_h2))
        else:
            raise ValueError(kind)
        bs.append(torch.from_numpy(np.ascontiguousarray(s.b, dtype=np.float64)).to(device))
        xs.append(torch.zeros(n, dtype=torch.float64, device=device))
    return ops, bs, xs
