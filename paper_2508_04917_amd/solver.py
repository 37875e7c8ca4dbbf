"""Convenience layer: upload a BSR problem and run the library's setup.

Only device-memory plumbing (torch tensors) and calls into the C ABI."""

from __future__ import annotations

import numpy as np
import torch

from . import ddilu as dd


class DDSolver:
    """Partition + factor a BSR matrix on the GPU and keep the handle."""

    def __init__(self, nx, ny, nz, bs, brow_ptr, bcol, val, sub=(0, 0, 0), precision=dd.DD_FP64,
                 n_cu=0, lds_budget_bytes=0, device="cuda", graph_part_rows=None):
        """graph_part_rows: None for geometric cuts of the nx*ny*nz grid;
        otherwise partition the matrix graph (no geometry) into parts of that
        many rows (0 = automatic)."""
        self.device = device
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dt).reshape(-1)
        ptr_d = t(brow_ptr, torch.int32)
        col_d = t(bcol, torch.int32)
        val_d = t(val, torch.float64)
        if graph_part_rows is None:
            self.h = dd.dd_partition(nx, ny, nz, bs, ptr_d, col_d, val_d, sub=sub, n_cu=n_cu,
                                     lds_budget_bytes=lds_budget_bytes)
        else:
            self.h = dd.dd_partition_graph(nx * ny * nz, bs, ptr_d, col_d, val_d, part_rows=graph_part_rows,
                                           lds_budget_bytes=lds_budget_bytes)
        del ptr_d, col_d, val_d
        dd.ilu0_factor(self.h, precision)
        self.info = dd.dd_get_info(self.h)
        self.n, self.bs = self.info["n"], self.info["bs"]

    @classmethod
    def from_problem(cls, p, sub=(0, 0, 0), precision=dd.DD_FP64, **kw):
        return cls(p.nx, p.ny, p.nz, p.bs, p.brow_ptr, p.bcol, p.val, sub=sub, precision=precision, **kw)

    def set_precision(self, precision):
        dd.dd_set_precision(self.h, precision)
        self.info = dd.dd_get_info(self.h)

    def apply(self, r, z=None):
        return dd.dd_trsv_apply(self.h, r, z)

    def spmv(self, x, y=None):
        return dd.dd_spmv(self.h, x, y)

    def solve(self, b, x=None, rtol=1e-8, maxit=10000):
        return dd.bicgstab_solve(self.h, b, x, rtol=rtol, maxit=maxit)

    def close(self):
        self.h.close()
