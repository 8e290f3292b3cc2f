"""Pins of the paper-layout 4-D table (Sec. II.F, III.A) in the oracle."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from conftest import rel_err
from oracle import physics as P
from oracle import table4d as T4
from oracle.tables import Axis


def test_nodes_are_the_bridged_closed_form_everywhere_on_the_paper_ranges():
    ax = T4.paper_axes(8)
    tab = T4.build(ax)
    assert np.all(np.isfinite(tab))
    # against the printed form of the bridge (the oracle's rates use the rewritten form)
    rng = np.random.default_rng(4)
    idx = rng.integers(0, 8, size=(50, 4))
    H, B, n_e, T_e = (10.0 ** ax[d].nodes()[idx[:, d]] for d in range(4))
    r = P.direct_rates(n_e, T_e, T_e, B, H)
    printed = P.hubeny_total(r["q_thin"], T_e, H, P.tau_scattering(n_e, H))
    assert np.max(rel_err(2.0 ** tab[tuple(idx.T)], printed)) < 1e-11


def test_interp4_reproduces_multilinear_functions_and_nodes():
    ax = (Axis(5, 0.0, 4.0), Axis(6, -1.0, 1.5), Axis(4, 2.0, 3.0), Axis(7, 10.0, 13.0))
    g = np.meshgrid(*[np.arange(a.n, dtype=float) for a in ax], indexing="ij")
    # sum of products of one index per axis pair is multilinear: reproduced exactly
    f = lambda i0, i1, i2, i3: 1.5 + 0.3 * i0 - 2.0 * i1 * i3 + 0.7 * i2 * i0 + 0.1 * i0 * i1 * i2 * i3
    tab = f(*g)
    rng = np.random.default_rng(1)
    u = [rng.uniform(a.lo, a.hi, 500) for a in ax]
    y, cl = T4.interp4(tab, ax, u)
    fi = [(v - a.lo) / a.step for v, a in zip(u, ax)]
    assert np.max(np.abs(y - f(*fi))) < 1e-12 and not cl.any()
    nodes = [a.nodes()[[0, a.n - 1, 2]] for a in ax]
    y, _ = T4.interp4(tab, ax, nodes)
    assert np.max(np.abs(y - tab[(0, ax[0].n - 1, 2), (0, ax[1].n - 1, 2), (0, ax[2].n - 1, 2),
                                 (0, ax[3].n - 1, 2)])) < 1e-12
    y, cl = T4.interp4(tab, ax, [np.array([a.lo - 1.0]) for a in ax])
    assert cl.all() and abs(y[0] - tab[0, 0, 0, 0]) < 1e-12


def test_interp4_matches_scipy():
    ax = (Axis(5, 0.0, 4.0), Axis(6, -1.0, 1.5), Axis(4, 2.0, 3.0), Axis(7, 10.0, 13.0))
    tab = np.random.default_rng(2).normal(size=tuple(a.n for a in ax))
    rgi = RegularGridInterpolator([a.nodes() for a in ax], tab)
    rng = np.random.default_rng(3)
    u = [rng.uniform(a.lo, a.hi, 400) for a in ax]
    y, _ = T4.interp4(tab, ax, u)
    assert np.max(np.abs(y - rgi(np.stack(u, axis=1)))) < 1e-12
