"""Write tests/golden/ode_reference_iid2m_256.json: the cooling ODE integrated
to tight tolerance (the oracle's stiff Radau integration, rtol 1e-11) over one
step dt = 1e-3 r_g/c for 256 seeded cells of the 2^21-cell iid workload, with
the oracle's own FP64 64^3 tables.  It is the reference against which the
backward-Euler and explicit 16-substep updates are compared (model accuracy of
the two time integrators, not a parity check).  Calls only the oracle.

    python tests/golden/make_ode_reference.py
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import finegrid as F  # noqa: E402
from oracle import step as S  # noqa: E402
from oracle import tables as T  # noqa: E402
from paper_2505_08855_amd import workloads as W  # noqa: E402

N_CELLS = 256
WORKLOAD = 3
OUT = os.path.join(HERE, "ode_reference_iid2m_256.json")
_TS = None


def _init():
    global _TS
    spec = T.TableSpec.default(64)
    _TS = S.TableSet(spec, T.build_tables(spec))


def _one(cell):
    return F.integrate_ode(_TS, cell, W.DT_DEFAULT)


def main():
    cells = W.workload(WORKLOAD)
    n = cells["n_e"].size
    idx = np.sort(np.random.default_rng(W.SEED_BASE + 100).choice(n, size=N_CELLS, replace=False))
    rows = [[float(cells[f][i]) for f in W.FIELDS] for i in idx]
    with Pool(min(8, os.cpu_count() or 1), initializer=_init) as pool:
        res = pool.map(_one, rows)
    doc = {"description": "cooling ODE over one step (oracle Radau, rtol 1e-11, FP64 64^3 tables), "
                          "256 seeded cells of workload %d (iid 2^21)" % WORKLOAD,
           "dt": W.DT_DEFAULT, "workload": WORKLOAD, "index": [int(i) for i in idx],
           "fields": list(W.FIELDS), "cells": rows,
           "T_e_ode": [r[0] for r in res], "T_i_ode": [r[1] for r in res]}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=0)
    print(OUT)


if __name__ == "__main__":
    main()
