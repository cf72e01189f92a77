"""dtau -> 0 estimates: the same impurities solved at several numbers of time
slices in one uneven-L batch, then a weighted fit even in dtau
(hfqmc_extrapolate) per impurity and observable."""
from __future__ import annotations

import numpy as np

from . import hfqmc


def solve_extrapolated(ctx: hfqmc.Context, problems_by_L: dict, order: int = 1,
                       keys=("n_up", "n_dn", "docc")):
    """problems_by_L maps L -> list of problem dicts (the same impurities in
    the same order at each L).  Returns (list of dicts {key: c0, key_err: err
    of c0}, per-L solver results)."""
    Ls = sorted(problems_by_L)
    n = len(problems_by_L[Ls[0]])
    if any(len(problems_by_L[L]) != n for L in Ls):
        raise ValueError("every L needs the same impurities")
    batch = [p for L in Ls for p in problems_by_L[L]]
    res = ctx.solve(batch)
    per_L = {L: res[k * n:(k + 1) * n] for k, L in enumerate(Ls)}
    out = []
    for i in range(n):
        d = [problems_by_L[L][i]["beta"] / L for L in Ls]
        row = {}
        for key in keys:
            c, ce = hfqmc.extrapolate(d, [per_L[L][i][key] for L in Ls], [per_L[L][i][key + "_err"] for L in Ls],
                                      order)
            row[key], row[key + "_err"] = float(c[0]), float(ce[0])
        out.append(row)
    return out, per_L
