"""Write the "oracle_table2_record" block of paper_tables_1_2.json.

These are not paper values: they record what the oracle's smoother reading
(node-star multiplicative Schwarz + l1-Jacobi) gives on the Table 2 stripes
workload for the refinement-based (Ref) and geometric (Geo) hierarchies,
which the printed Table 2 does not match.  Calls only oracle/ and gen/.

    python tests/golden/record_table2.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

import numpy as np  # noqa: E402

import gen  # noqa: E402
import oracle  # noqa: E402
from gen import fields  # noqa: E402
from refsel import RefSelector  # noqa: E402


def run(L, interp, schwarz, smoother="stars", stripes=True):
    alpha = (lambda m: fields.stripes_2d(m)) if stripes else 1.0
    p = gen.make_problem("tri", L, beta=0.01, alpha=alpha)
    n = p.A.shape[0]
    b = np.arange(1, n + 1, dtype=float)
    x0 = np.random.default_rng(0).random(n)
    if interp == "ref":
        H = oracle.setup(p.A, p.G, interp="ref", ref_select=RefSelector(p), max_levels=L,
                         min_coarse=0, schwarz=schwarz, smoother_blocks=smoother)
    elif interp == "alg":
        H = oracle.setup(p.A, p.G, schwarz=schwarz, smoother_blocks=smoother)
    else:
        H = oracle.setup(p.A, p.G, user=gen.geo_hierarchy("tri", L, L), schwarz=schwarz)
    _, it, _ = oracle.pcg(H, p.A, b, x0=x0)
    _, ita, h = oracle.amg_solve(H, p.A, b, x0=x0)
    return it, ita, round(float(h[-1] / h[-2]), 4)


def main():
    path = os.path.join(HERE, "paper_tables_1_2.json")
    g = json.load(open(path))
    rec = {"source": g.get("oracle_table2_record", {}).get("source", "")}
    for L in (4, 5):
        rec[str(L)] = {}
        for interp in ("ref", "geo"):
            it, _, _ = run(L, interp, "adjoint")
            _, ita, conv = run(L, interp, "repeat")
            rec[str(L)][interp] = {"pcg": it, "amg": ita, "amg_conv": conv}
    g["oracle_table2_record"] = rec
    # the alternative reading: node stars plus the interior blocks of each
    # level's splitting; Table 2 (stripes) and Table 1 (isotropic)
    rec2 = {"source": g.get("oracle_record_stars_interior", {}).get("source", "")}
    for L in (4, 5):
        rec2[str(L)] = {}
        for interp in ("ref", "alg"):
            for tab, stripes in (("table2", True), ("table1", False)):
                it, _, _ = run(L, interp, "adjoint", "stars+interior", stripes)
                _, ita, conv = run(L, interp, "repeat", "stars+interior", stripes)
                rec2[str(L)][f"{tab}_{interp}"] = {"pcg": it, "amg": ita, "amg_conv": conv}
    g["oracle_record_stars_interior"] = rec2
    json.dump(g, open(path, "w"), indent=1)


if __name__ == "__main__":
    main()
