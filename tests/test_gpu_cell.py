"""GPU parity of the cell-blocked table layout (variant "cell").

The variant reads a copy of the FP32 tables in which the 8 corners of every
table cell sit together (one 128-byte line per cooling cell).  The corner
values are the same floats and the per-cell arithmetic is that of the GLOBAL
variant, compiled once per accessor, so values agree to rounding (1e-12) and
statuses exactly; the energy tier against the oracle holds on its own.
"""
import numpy as np
import pytest

from conftest import rel_err
from oracle import step as S
from oracle import tables as T
from paper_2505_08855_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2505_08855_amd.radcool")
DT = W.DT_DEFAULT
OUT_KEYS = ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "Q_brem", "Q_syn", "eta")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def imported64(dev, tables64):
    co, re, stored = T.quantize_tables(tables64)
    resid = np.concatenate([re[k].ravel() for k in T.TABLE_NAMES])
    coeffs = np.stack([co[k] for k in T.TABLE_NAMES])
    return R.Tables.from_storage(R.default_spec(64), resid, coeffs), stored


def to_dev(cells, dev):
    return {k: torch.from_numpy(np.ascontiguousarray(cells[k], dtype=np.float64)).to(dev) for k in W.FIELDS}


def run(gt, st, dt, **kw):
    out = R.cool_step(gt, st, dt, R.default_opts(**kw), diagnostics=True)
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def assert_same(a, b):
    assert np.array_equal(a["status"], b["status"])
    for k in OUT_KEYS:
        both_nan = np.isnan(a[k]) & np.isnan(b[k])
        err = rel_err(a[k], b[k])
        assert np.all(both_nan | (err < 1e-12)), (k, float(np.nanmax(err)))


@pytest.mark.parametrize("scheme", ["newton", "explicit16", "rates"])
@pytest.mark.parametrize("shape", ["iid", "sphere"])
def test_cell_equals_global(dev, imported64, scheme, shape):
    gt, _ = imported64
    cells = W.workload(0, n=100_003) if shape == "iid" else W.sphere_cells(n_r=16, n_th=16, n_ph=256)
    st = to_dev(cells, dev)
    dt = DT * 1e3 if scheme == "newton" else DT
    assert_same(run(gt, st, dt, scheme=scheme, variant="cell"), run(gt, st, dt, scheme=scheme, variant="global"))


@pytest.mark.parametrize("n", [1, 63, 4099])
def test_cell_energy_tier(dev, imported64, spec64, n):
    """The Newton step through the cell-blocked copy against the oracle's
    backward Euler on the same stored tables (ragged sizes, stiff step)."""
    gt, stored = imported64
    cells = W.workload(3, n=n)
    dt = DT * 1e3
    out = run(gt, to_dev(cells, dev), dt, variant="cell")
    ref = S.step_be(S.TableSet(spec64, stored), *[cells[f] for f in W.FIELDS], dt)
    assert np.array_equal(out["status"], ref["status"])
    for k in ("T_e_new", "T_i_new"):
        assert np.max(rel_err(out[k], ref[k])) < 1e-9, k


def test_cell_full_size_matches_global(dev):
    """256^3 independent cells on 128^3 tables, the bench's launch: every cell
    agrees with the GLOBAL variant."""
    gt = R.Tables.build(R.default_spec(128))
    cells = W.workload(1)
    st = to_dev(cells, dev)
    a = R.cool_step(gt, st, DT, R.default_opts(variant="cell"))
    b = R.cool_step(gt, st, DT, R.default_opts(variant="global"))
    assert torch.equal(a["status"], b["status"])
    for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc"):
        err = ((a[k] - b[k]).abs() / b[k].abs().clamp_min(1e-300)).max().item()
        assert err < 1e-12, (k, err)
    gt.destroy()


def test_cell_rejects_bf16_tables_and_empty_is_noop(dev):
    gt = R.Tables.build(R.default_spec(16, "bf16"))
    st = to_dev(W.workload(0, n=64), dev)
    with pytest.raises(R.RadcoolError):
        R.cool_step(gt, st, DT, R.default_opts(variant="cell"))
    gt.destroy()
    gt = R.Tables.build(R.default_spec(16))
    z = {k: torch.empty(0, dtype=torch.float64, device=dev) for k in W.FIELDS}
    assert R.cool_step(gt, z, DT, R.default_opts(variant="cell"))["T_e_new"].numel() == 0
    # the first non-empty call builds the copy, later calls reuse it
    a = run(gt, st, DT, variant="cell")
    b = run(gt, st, DT, variant="cell")
    assert_same(a, b)
    gt.destroy()
