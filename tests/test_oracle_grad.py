"""Pins of the oracle's gradient (oracle/grad.py) by central finite differences
of the oracle's own forward step.  CPU only.

Finite differences through an implicit solve are limited by the solve's
rounding (a few ulps of T'), so every comparison carries a noise allowance
computed from the magnitude of the cell's loss terms; cells whose
perturbation moves any table coordinate into another cell are skipped (the
interpolant is only piecewise smooth).
"""
import numpy as np
import pytest

from oracle import grad as Gd
from oracle import step as S
from oracle import tables as T
from oracle.tables import axis_coord
from paper_2505_08855_amd import workloads as W

DT = W.DT_DEFAULT
F = W.FIELDS


@pytest.fixture(scope="module")
def setup(ts64):
    cells = W.workload(0, n=384)
    out = S.step_be(ts64, *[cells[f] for f in F], DT)
    rng = np.random.default_rng(11)
    n = cells["n_e"].size
    g = {k: rng.normal(size=n) for k in ("te", "ti", "qr", "qc")}
    G = Gd.vjp_step_be(ts64, cells, out, DT, g["te"], g["ti"], g["qr"], g["qc"])
    return cells, out, g, G


def loss_cells(out, g):
    return g["te"] * out["T_e_new"] + g["ti"] * out["T_i_new"] + g["qr"] * out["q_rad"] + g["qc"] * out["q_cc"]


def magnitude(out, g):
    return (np.abs(g["te"] * out["T_e_new"]) + np.abs(g["ti"] * out["T_i_new"])
            + np.abs(g["qr"] * out["q_rad"]) + np.abs(g["qc"] * out["q_cc"]))


def cell_indices(spec, c, o):
    ne, te, ti, B, H = (c[f] for f in F)
    us = [(np.log10(ne) + np.log10(H), spec.cool[0]), (np.log10(te), spec.cool[1]), (np.log10(B), spec.cool[2]),
          (np.log10(ne), spec.coul[0]), (np.log10(te), spec.coul[1]), (np.log10(ti), spec.coul[2]),
          (np.log10(o["T_e_new"]), spec.cool[1]), (np.log10(o["T_e_new"]), spec.coul[1]),
          (np.log10(o["T_i_new"]), spec.coul[2])]
    return np.stack([axis_coord(u, a)[0] for u, a in us])


@pytest.mark.parametrize("field", F)
def test_input_gradients_match_central_differences(ts64, spec64, setup, field):
    cells, out, g, G = setup
    h = 1e-6
    cp, cm = dict(cells), dict(cells)
    cp[field] = cells[field] * (1 + h)
    cm[field] = cells[field] * (1 - h)
    op = S.step_be(ts64, *[cp[f] for f in F], DT)
    om = S.step_be(ts64, *[cm[f] for f in F], DT)
    fd = (loss_cells(op, g) - loss_cells(om, g)) / (2 * h * cells[field])
    same = np.all(cell_indices(spec64, cp, op) == cell_indices(spec64, cm, om), axis=0)
    same &= op["status"] == om["status"]
    assert same.sum() > 300
    noise = 1e-13 * magnitude(out, g) / (2 * h * cells[field])
    err = np.abs(fd - G[field])
    assert np.all((err <= 1e-6 * np.abs(G[field]) + noise)[same])


def test_table_gradients_match_central_differences(ts64, spec64, tables64, setup):
    cells, out, g, G = setup
    d = 1e-5
    L0 = magnitude(out, g)
    # the table entries each cell reads: input state and solution
    parts = []
    for x, z in ((cells["T_e"], cells["T_i"]), (out["T_e_new"], out["T_i_new"])):
        uN = np.log10(cells["n_e"]) + np.log10(cells["H"])
        _, _, ic, _ = Gd.interp_parts(tables64["brem"], spec64.cool, uN, np.log10(x), np.log10(cells["B"]))
        _, _, ik, _ = Gd.interp_parts(tables64["coul"], spec64.coul, np.log10(cells["n_e"]), np.log10(x),
                                      np.log10(z))
        parts.append((ic, ik))
    for name in T.TABLE_NAMES:
        which = 1 if name == "coul" else 0
        size = tables64[name].size
        noise = np.zeros(size)
        for p in parts:
            np.add.at(noise, p[which].ravel(), np.repeat(1e-13 * L0 / (2 * d), 8))
        gt = G["tables"][name].ravel()
        score = np.abs(gt) / np.maximum(noise, 1e-300)
        picks = [k for k in np.argsort(score)[::-1][:4] if score[k] > 1e4]
        assert picks, name
        for k in picks:
            tp = {kk: v.copy() for kk, v in tables64.items()}
            tm = {kk: v.copy() for kk, v in tables64.items()}
            tp[name].ravel()[k] += d
            tm[name].ravel()[k] -= d
            lp = loss_cells(S.step_be(S.TableSet(spec64, tp), *[cells[f] for f in F], DT), g)
            lm = loss_cells(S.step_be(S.TableSet(spec64, tm), *[cells[f] for f in F], DT), g)
            fd = np.sum(lp - lm) / (2 * d)
            assert abs(fd - gt[k]) <= 1e-6 * abs(gt[k]) + 10 * noise[k], (name, k, fd, gt[k])


def test_floor_cells_gradient(ts64, spec64):
    """On a floor-projected cell T_e' is constant: its cotangent has no effect."""
    c = {"n_e": np.array([1e20]), "T_e": np.array([2e6]), "T_i": np.array([2e6]),
         "B": np.array([1e8]), "H": np.array([1e4])}
    out = S.step_be(ts64, *[c[f] for f in F], 1e3 * DT, T_floor=1.5e6)
    assert out["status"][0] & S.ST_FLOOR
    G = Gd.vjp_step_be(ts64, c, out, 1e3 * DT, 1.0, 0.0, T_floor=1.5e6)
    for f in F:
        assert G[f][0] == 0.0
    # d T_i' / d T_i by finite differences (strong coupling makes it ~5e-6, so
    # a larger step keeps the bisection's rounding of T_i' out of the quotient)
    h = 1e-4
    cp, cm = dict(c), dict(c)
    cp["T_i"] = c["T_i"] * (1 + h)
    cm["T_i"] = c["T_i"] * (1 - h)
    op = S.step_be(ts64, *[cp[f] for f in F], 1e3 * DT, T_floor=1.5e6)
    om = S.step_be(ts64, *[cm[f] for f in F], 1e3 * DT, T_floor=1.5e6)
    fd = (op["T_i_new"][0] - om["T_i_new"][0]) / (2 * h * c["T_i"][0])
    G2 = Gd.vjp_step_be(ts64, c, out, 1e3 * DT, 0.0, 1.0, T_floor=1.5e6)
    assert G2["T_i"][0] == pytest.approx(fd, rel=1e-4)
