"""The shapes of the paper's structured test matrices (Section 5.3, Table 5):
laplacian1 (128^3) and laplacian2 (128x128x256) as 3x3 BSR Laplacians cut
into 8x16x16 boxes of 2,048 block rows, set up on the GPU.  The counts the
paper prints (scalar nonzeros before and after the drop, in
tests/golden/table5_partition.txt) must come out of the library's own
partition and drop, and the preconditioned solve must converge."""

import os

import numpy as np
import pytest

from problems import laplacian_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table5_partition.txt")


def rows():
    out = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                out.append((t[0],) + tuple(int(v) for v in t[1:]))
    return out


@pytest.mark.parametrize("row", rows(), ids=lambda r: r[0])
def test_table5_shapes_on_gpu(row):
    name, nx, ny, nz, sx, sy, sz, nsub, nnz_full, nnz_drop = row
    print(f"[table5] {name}: {nx}x{ny}x{nz} 3x3 blocks, subdomains {sx}x{sy}x{sz}", flush=True)
    p = laplacian_blocks(nx, ny, nz, seed=31)
    s = DDSolver.from_problem(p, sub=(sx, sy, sz))
    inf = s.info
    print(f"[table5] {name}: {inf['nsub']} subdomains, {inf['nnzb']} blocks, {inf['nnzb_dropped']} after the drop",
          flush=True)
    assert inf["nsub"] == nsub
    assert 9 * inf["nnzb"] == nnz_full
    assert 9 * inf["nnzb_dropped"] == nnz_drop
    b = torch.as_tensor(p.b, device="cuda")
    x, info = s.solve(b, rtol=1e-8, maxit=5000)
    print(f"[table5] {name}: BiCGSTAB {info['iters']} iterations, true residual {info['rel_res_true']:.2e}",
          flush=True)
    assert info["status"] == dd.DD_OK and info["rel_res_true"] <= 2e-8
    s.close()
