"""GPU parity of the bfloat16 table storage form (storage-precision experiment).

  * build: the GPU-built residuals are bfloat16 values and equal the oracle's
    bfloat16 storage form of its FP64 tables up to one bfloat16 step (the two
    node evaluations differ at 1e-13, which can move a rounding decision);
  * energies on identical (imported) bfloat16 tables: 1e-9, as for FP32;
  * rates against the oracle's unrounded FP64 tables: within the storage
    bound ln 2 * max|residual| * 2^-8 of each table (half a bfloat16 step of
    the largest residual, as a relative error of 2^y; Q_rad adds the synch
    and eta bounds, its bridge factor being at most 1), plus the FP32 tier.
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


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return torch.device("cuda:0")


def to_dev(cells, dev):
    return {k: torch.from_numpy(np.ascontiguousarray(cells[k], dtype=np.float64)).to(dev) for k in W.FIELDS}


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


@pytest.fixture(scope="module")
def bf16_storage(tables64):
    co, re, st = T.quantize_tables(tables64, "bf16")
    resid = np.concatenate([re[k].ravel() for k in T.TABLE_NAMES])
    coeffs = np.stack([co[k] for k in T.TABLE_NAMES])
    return resid, coeffs, st


@pytest.fixture(scope="module")
def cells0():
    return W.workload(0)


def test_bf16_build_matches_oracle_storage(dev, bf16_storage):
    gt = R.Tables.build(R.default_spec(64, "bf16"))
    resid, coeffs = gt.export()
    assert np.array_equal(T.round_bf16(resid), resid)
    ref, ref_co, _ = bf16_storage
    assert np.max(np.abs(coeffs - ref_co)) < 1e-9
    # one bfloat16 step is at most 2^-7 of the value
    assert np.all(np.abs(resid - ref) <= np.abs(ref) * 2.0 ** -7 + 1e-30)
    assert np.mean(resid == ref) > 0.999


def test_bf16_energy_tier(dev, spec64, bf16_storage, cells0):
    resid, coeffs, stored = bf16_storage
    gt = R.Tables.from_storage(R.default_spec(64, "bf16"), resid, coeffs)
    got_resid, _ = gt.export()
    assert np.array_equal(got_resid, resid)
    out = to_np(R.cool_step(gt, to_dev(cells0, dev), DT))
    ref = S.step_be(S.TableSet(spec64, stored), *[cells0[f] for f in W.FIELDS], DT)
    for k in ("T_e_new", "T_i_new"):
        assert np.max(rel_err(out[k], ref[k])) < 1e-9, k
    assert np.array_equal(out["status"], ref["status"])


def test_bf16_rates_within_storage_bound(dev, ts64, bf16_storage, cells0):
    gt = R.Tables.build(R.default_spec(64, "bf16"))
    resid, _ = gt.export()
    vc = 64 ** 3
    amax = [np.max(np.abs(resid[k * vc:(k + 1) * vc])) for k in range(4)]
    bound = [np.log(2.0) * a * 2.0 ** -8 + 1e-5 for a in amax]
    out = to_np(R.cool_step(gt, to_dev(cells0, dev), DT, R.default_opts(scheme="rates"), diagnostics=True))
    ref = S.table_rates(ts64, *[cells0[f] for f in W.FIELDS])
    ok = (ref["status"] & 1) == 0
    checks = (("Q_brem", "q_brem", bound[0]), ("Q_syn", "q_syn", bound[1]), ("eta", "eta", bound[2]),
              ("Q_cc", "q_cc", bound[3]), ("Q_rad", "q_rad", max(bound[0], bound[1] + bound[2])))
    for g, r, b in checks:
        e = rel_err(out[g][ok], ref[r][ok])
        assert np.max(e) <= b, (g, np.max(e), b)
