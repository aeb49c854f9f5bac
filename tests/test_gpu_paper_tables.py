"""The paper's data-free iteration studies, run through the GPU path (the studies need no
dataset: constant medium, 10 points per wavelength, J = n/10, residual reduction 1e-6).

Table 4 (Sec. 4.4), PML column: 2-D unit square, n = 100 ... 1600, one point source at the
centre of the padded grid, outer PML 10 cells, interface PML 8 cells (the widths the
oracle's pin uses), complex128.  Table 3 (Sec. 4.3): 3-D unit cube, slabs of 10 planes,
interface PML width w_pml = 3 ... 6 (outer PML of the same width): 100^3 in complex128,
200^3 in mixed precision (its complex128 slab inverses would not fit in HBM at w_pml = 6;
the mixed path's restart from P r counts one extra iteration).  The paper does not state
its PML profile, so these are soft pins."""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DEV = "cuda:0"
TABLE4 = json.load(open(os.path.join(HERE, "golden", "table4_pml_const2d.json")))["rows"]
TABLE3 = json.load(open(os.path.join(HERE, "golden", "table3_pml_const3d.json")))["rows"]


@pytest.mark.parametrize("row", TABLE4, ids=[f"n{r['n']}" for r in TABLE4])
def test_table4_pml_column(row):
    from paper_1208_3956_amd import Helmholtz
    n, J = row["n"], row["J"]
    h = 1.0 / n
    H = Helmholtz(np.ones((n, n)), 2 * math.pi / (10 * h), h, J, pml_outer=10, pml_iface=8,
                  prec="c128", mode="reduced", device=DEV).factor()
    f = torch.zeros((1, H.N_y, H.N_x), dtype=torch.complex128, device=DEV)
    f[0, H.N_y // 2, H.N_x // 2] = 1.0 / h ** 2
    res = H.solve(f, 1e-6)
    H.close()
    print(f"Table 4 n={n} J={J}: {res.iters[0]} iterations (paper: {row['iterations']})", flush=True)
    assert res.status == 0 and res.relres[0] <= 1e-6
    assert abs(res.iters[0] - row["iterations"]) <= 1


def _table3(n, J, w, prec):
    from paper_1208_3956_amd import Helmholtz
    h = 1.0 / n
    H = Helmholtz(np.ones((n, n, n)), 2 * math.pi / (10 * h), h, J, pml_outer=w, pml_iface=w,
                  prec=prec, mode="reduced", device=DEV).factor()
    f = torch.zeros((1, H.N_z, H.N_y, H.N_x), dtype=torch.complex128, device=DEV)
    f[0, H.N_z // 2, H.N_y // 2, H.N_x // 2] = 1.0 / h ** 3
    res = H.solve(f, 1e-6)
    slots, path = H.factor_slots, H.factor_path
    H.close()
    return res, slots, path


@pytest.mark.parametrize("w", [3, 4, 5, 6])
def test_table3_const3d_100(w):
    row = TABLE3[0]
    res, slots, path = _table3(row["n"], row["J"], w, "c128")
    want = row["w_pml"][str(w)]
    print(f"Table 3 n={row['n']} J={row['J']} w_pml={w}: {res.iters[0]} iterations (paper: {want}), "
          f"{slots} factorisations", flush=True)
    # a constant medium: the interior slabs share one factorisation (Sec. 4.3)
    assert slots == 3
    assert res.status == 0 and res.relres[0] <= 1e-6
    assert abs(res.iters[0] - want) <= 1


@pytest.mark.parametrize("w", [3, 4, 5, 6])
def test_table3_const3d_200(w):
    row = TABLE3[1]
    res, slots, path = _table3(row["n"], row["J"], w, "mixed")
    want = row["w_pml"][str(w)]
    print(f"Table 3 n={row['n']} J={row['J']} w_pml={w}: {res.iters[0]} iterations (paper: {want}), "
          f"{slots} factorisations, factor path {path}", flush=True)
    assert slots == 3
    assert res.status == 0 and res.relres[0] <= 1e-6
    assert -1 <= res.iters[0] - want <= 2
