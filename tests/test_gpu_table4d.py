"""GPU parity of the paper-layout 4-D table (Sec. II.F, III.A): node values
against the oracle's closed forms (FP32 storage of log2 values), rates on
identical (imported) values against the oracle's interpolation."""
import numpy as np
import pytest

from conftest import rel_err
from oracle import table4d as T4
from paper_2505_08855_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2505_08855_amd.radcool")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return torch.device("cuda:0")


def axes_of(ax):
    a = R.Axes4()
    for d, x in enumerate(ax):
        a.n[d], a.lo[d], a.hi[d] = x.n, x.lo, x.hi
    return a


def test_table4d_build_matches_oracle_nodes(dev):
    ax = T4.paper_axes(16)
    t = R.Table4D.build(axes_of(ax))
    _, v = t.export()
    ref = T4.build(ax)
    # FP32 storage of log2 values: half an ulp of |y| (up to ~170) plus evaluation differences
    assert np.all(np.abs(v - ref) <= np.abs(ref) * 2.0 ** -24 + 1e-8)


def test_full_paper_table_builds(dev):
    """The paper's 100^4 table at full size: 4000 seeded nodes against the
    oracle's closed forms at those nodes (log2 of the bridged Q_total, FP32
    storage), plus the host build of the same nodes."""
    t = R.Table4D.build()            # 100^4 nodes, 400 MB
    a, v = t.export()
    assert list(a.n) == [100] * 4 and np.all(np.isfinite(v))
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 100, size=(4000, 4))
    ax = T4.paper_axes(100)
    H, B, n_e, T = (10.0 ** ax[d].nodes()[idx[:, d]] for d in range(4))
    got = v[tuple(idx.T)].astype(np.float64)
    ref = np.log2(T4.physics.direct_rates(n_e, T, T, B, H)["q_rad"])
    assert np.all(np.abs(got - ref) <= np.abs(ref) * 2.0 ** -24 + 1e-8)
    host = R.selftest_node4d_host(H, B, n_e, T)
    assert np.max(np.abs(got - host) - np.abs(host) * 2.0 ** -24) < 1e-8


@pytest.mark.parametrize("n", [1, 4097, 262_147])
def test_rates4d_on_identical_values(dev, n):
    ax = T4.paper_axes(12)
    tab = T4.build(ax).astype(np.float32)
    t = R.Table4D.from_values(axes_of(ax), tab)
    cells = W.workload(0, n=n)
    st = {k: torch.from_numpy(np.ascontiguousarray(cells[k])).to(dev) for k in W.FIELDS}
    q, s = R.rates4d(t, st)
    q = q.cpu().numpy()
    ref = T4.q_total(tab.astype(np.float64), ax, cells["n_e"], cells["T_e"], cells["B"], cells["H"])
    ref = np.where(cells["T_e"] < 1e6, 0.0, ref)
    assert np.max(rel_err(q, ref)) < 1e-12
    assert np.all(s.cpu().numpy() == 0)
