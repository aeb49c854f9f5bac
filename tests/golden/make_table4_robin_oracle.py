"""Writes table4_robin_oracle.json: the iteration counts of the oracle's Robin-transmission
double sweep (Sec. 4.4) on the problems of Table 4 (constant medium on the unit square,
N_x = N_y = n, h = 1/n, 10 points per wavelength, J = n/10, a point source 1/h^2 at the
centre of the padded grid, outer PML 10 cells, unrestarted GMRES to a residual reduction of
1e-6).  With --concurrent it writes table4_concurrent_robin_oracle.json instead: the same
problems up to n = 800 with the concurrent Robin sweeps of Sec. 3.1.  Calls nothing but the
oracle.  Run from the repository root:
    python tests/golden/make_table4_robin_oracle.py [--concurrent]
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.grid import make_geometry  # noqa: E402
from oracle.solve import solve_dd_concurrent_robin, solve_dd_robin  # noqa: E402


def main():
    concurrent = "--concurrent" in sys.argv[1:]
    solve, name, out_name = ((solve_dd_concurrent_robin, "solve_dd_concurrent_robin",
                              "table4_concurrent_robin_oracle.json") if concurrent else
                             (solve_dd_robin, "solve_dd_robin", "table4_robin_oracle.json"))
    paper = json.load(open(os.path.join(HERE, "table4_robin_const2d.json")))["rows"]
    rows = []
    for row in paper:
        n, J = row["n"], row["J"]
        if concurrent and n > 800:
            break
        h = 1.0 / n
        t0 = time.time()
        g = make_geometry(np.ones((n, n)), 2 * math.pi / (10 * h), h, 10, 8, J)
        f = np.zeros((g.N_y, g.N_x), complex)
        f[g.N_y // 2, g.N_x // 2] = 1 / h ** 2
        res = solve(g, f, 1e-6)
        rows.append({"n": n, "J": J, "iterations": int(res.iters), "relres": float(res.relres)})
        print(f"n={n} J={J}: {res.iters} iterations (paper, Robin double sweep: {row['iterations']}), "
              f"{time.time() - t0:.0f} s", flush=True)
    out = {"source": f"oracle.solve.{name}, written by make_table4_robin_oracle.py",
           "problem": "Table 4 (Sec. 4.4): unit square, c = 1, 10 points per wavelength, J = n/10, "
                      "centre point source, outer PML 10 cells, tolerance 1e-6",
           "rows": rows}
    with open(os.path.join(HERE, out_name), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
