"""The paper's data-free iteration studies, run through the GPU path (the studies need no
dataset: constant medium, 10 points per wavelength, J = n/10, residual reduction 1e-6).

Table 4 (Sec. 4.4), PML column: 2-D unit square, n = 100 ... 1600, one point source at the
centre of the padded grid, outer PML 10 cells, interface PML 8 cells (the widths the
oracle's soft pin uses).  Table 3 (Sec. 4.3): 3-D unit cube, n = 100, slabs of 10 planes,
interface PML width w_pml = 3 ... 6 (outer PML of the same width).  The paper does not
state its PML profile, so these are soft pins: the counts may differ by up to two."""
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
    assert abs(res.iters[0] - row["iterations"]) <= 2


@pytest.mark.parametrize("w", [3, 4, 5, 6])
def test_table3_const3d_100(w):
    from paper_1208_3956_amd import Helmholtz
    row = TABLE3[0]
    n, J = row["n"], row["J"]
    h = 1.0 / n
    H = Helmholtz(np.ones((n, n, n)), 2 * math.pi / (10 * h), h, J, pml_outer=w, pml_iface=w,
                  prec="mixed", mode="reduced", device=DEV).factor()
    f = torch.zeros((1, H.N_z, H.N_y, H.N_x), dtype=torch.complex128, device=DEV)
    f[0, H.N_z // 2, H.N_y // 2, H.N_x // 2] = 1.0 / h ** 3
    res = H.solve(f, 1e-6)
    want = row["w_pml"][str(w)]
    print(f"Table 3 n={n} J={J} w_pml={w}: {res.iters[0]} iterations (paper: {want}), "
          f"factor path {H.factor_path}, {H.factor_slots} factorisations", flush=True)
    # a constant medium: the interior slabs share one factorisation (Sec. 4.3)
    assert H.factor_slots == 3
    H.close()
    assert res.status == 0 and res.relres[0] <= 1e-6
    assert abs(res.iters[0] - want) <= 2
