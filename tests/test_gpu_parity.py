"""GPU parity: the HIP path through the C ABI against the oracle.

Tiers (tolerances from the method's error budget):
  * table nodes: GPU-built log2 tables vs the oracle's FP64 build, 1e-6 relative
    in the tabulated value (FP32 storage of the residual plus build rounding);
  * rates: GPU tables + interpolation vs oracle FP64 tables + interpolation,
    1e-5 relative on Q_rad, Q_cc, Q_brem, Q_syn, eta;
  * energies: GPU Newton vs the oracle's backward-Euler solve on identical
    table data (the oracle's own tables in FP32 storage form, imported into the
    library), 1e-9 relative on T_e', T_i' (u = 1.5 n_e k T);
  * explicit update on identical tables: 1e-11.
"""
import os
import tempfile

import numpy as np
import pytest

from conftest import rel_err
from oracle import physics as P
from oracle import step as S
from oracle import tables as T
from paper_2505_08855_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2505_08855_amd.radcool")
DT = W.DT_DEFAULT
RATE_TOL = 1e-5
ENERGY_TOL = 1e-9


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return torch.device("cuda:0")


def to_dev(cells, dev, idx=None):
    out = {}
    for k in W.FIELDS:
        a = np.asarray(cells[k], dtype=np.float64)
        if idx is not None:
            a = a[idx]
        out[k] = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return out


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def storage_of(tables):
    co, re, st = T.quantize_tables(tables)
    resid = np.concatenate([re[k].ravel() for k in T.TABLE_NAMES])
    coeffs = np.stack([co[k] for k in T.TABLE_NAMES])
    return resid, coeffs, st


@pytest.fixture(scope="module")
def oracle128():
    spec = T.TableSpec.default(128)
    return spec, T.build_tables(spec)


@pytest.fixture(scope="module")
def cells0():
    return W.workload(0)


@pytest.fixture(scope="module")
def gpu_tables64(dev):
    return R.Tables.build(R.default_spec(64))


@pytest.fixture(scope="module")
def imported64(dev, tables64):
    resid, coeffs, stored = storage_of(tables64)
    return R.Tables.from_storage(R.default_spec(64), resid, coeffs), stored


def reconstruct(gt, spec):
    resid, coeffs = gt.export()
    vc = spec.cool.n[0] * spec.cool.n[1] * spec.cool.n[2]
    out = {}
    for k, name in enumerate(T.TABLE_NAMES):
        ax = spec.coul if k == 3 else spec.cool
        shape = tuple(ax.n)
        r = resid[k * vc: k * vc + int(np.prod(shape))].reshape(shape).astype(np.float64)
        g = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
        out[name] = coeffs[k, 0] + coeffs[k, 1] * g[0] + coeffs[k, 2] * g[1] + coeffs[k, 3] * g[2] + r
    return out


# ------------------------------------------------------------------ table build


def test_table_build_64_matches_oracle(gpu_tables64, tables64):
    got = reconstruct(gpu_tables64, R.default_spec(64))
    for name in T.TABLE_NAMES:
        # 1e-6 relative in the value is 1.44e-6 in log2
        assert np.max(np.abs(got[name] - tables64[name])) < 1.44e-6, name


def test_table_build_128_matches_oracle(dev, oracle128):
    gt = R.Tables.build(R.default_spec(128))
    got = reconstruct(gt, R.default_spec(128))
    for name in T.TABLE_NAMES:
        assert np.max(np.abs(got[name] - oracle128[1][name])) < 1.44e-6, name


# ------------------------------------------------------------------ rates tier


def test_rates_tier_config0(dev, gpu_tables64, ts64, cells0):
    out = to_np(R.cool_step(gpu_tables64, to_dev(cells0, dev), DT, R.default_opts(scheme="rates"),
                            diagnostics=True))
    ref = S.table_rates(ts64, *[cells0[f] for f in W.FIELDS])
    for g, r in (("Q_rad", "q_rad"), ("Q_cc", "q_cc"), ("Q_brem", "q_brem"), ("Q_syn", "q_syn"), ("eta", "eta")):
        e = rel_err(out[g], ref[r])
        assert np.max(e) < RATE_TOL, (g, np.max(e))
    assert np.array_equal(out["status"], ref["status"])


def test_direct_variant_matches_closed_forms(dev, cells0):
    idx = np.arange(0, 32768, 8)
    out = to_np(R.cool_step(R.Tables.build(R.default_spec(8)), to_dev(cells0, dev, idx), DT,
                            R.default_opts(scheme="rates", variant="direct"), diagnostics=True))
    ref = P.direct_rates(*[cells0[f][idx] for f in W.FIELDS])
    for g, r in (("Q_rad", "q_rad"), ("Q_cc", "q_cc"), ("Q_brem", "q_brem"), ("Q_syn", "q_syn"), ("eta", "eta")):
        assert np.max(rel_err(out[g], ref[r])) < 1e-9, g


# ------------------------------------------------------------------ energy tier


@pytest.fixture(scope="module")
def be_ref0(imported64, spec64, cells0):
    _, stored = imported64
    return S.step_be(S.TableSet(spec64, stored), *[cells0[f] for f in W.FIELDS], DT)


def test_energy_tier_config0(dev, imported64, cells0, be_ref0):
    gt, _ = imported64
    out = to_np(R.cool_step(gt, to_dev(cells0, dev), DT))
    for k in ("T_e_new", "T_i_new"):
        e = rel_err(out[k], be_ref0[k])
        assert np.max(e) < ENERGY_TOL, (k, np.max(e), int(np.argmax(e)))
    assert np.array_equal(out["status"], be_ref0["status"])
    assert np.max(rel_err(out["Q_rad"], be_ref0["q_rad"])) < 1e-12
    assert np.max(rel_err(out["Q_cc"], be_ref0["q_cc"])) < 1e-12


def test_explicit16_config0(dev, imported64, spec64, cells0):
    gt, stored = imported64
    out = to_np(R.cool_step(gt, to_dev(cells0, dev), DT, R.default_opts(scheme="explicit16")))
    ref = S.step_explicit16(S.TableSet(spec64, stored), *[cells0[f] for f in W.FIELDS], DT)
    for k in ("T_e_new", "T_i_new"):
        assert np.max(rel_err(out[k], ref[k])) < 1e-11, k


EDGE = {  # n_e, T_e, T_i, B, H
    "floor": (1e20, 2e6, 2e6, 1e8, 1e4),
    "heating": (1e16, 1e8, 1e11, 10.0, 1e6),
    "equal_T": (1e14, 1e9, 1e9, 1e4, 1e8),
    "T_e_above_T_i": (1e15, 1e10, 1e9, 1e4, 1e8),
    "clamped_low_n": (1e3, 1e8, 1e9, 1e2, 1e8),
    "clamped_high_T": (1e12, 3e12, 1e15, 1e6, 1e8),
    "below_floor": (1e12, 5e5, 2e5, 1e3, 1e8),
    "invalid_nan": (np.nan, 1e8, 1e9, 1e3, 1e8),
    "invalid_inf": (1e12, np.inf, 1e9, 1e3, 1e8),
    "invalid_neg": (1e12, -1e8, 1e9, 1e3, 1e8),
    "invalid_zero": (1e12, 1e8, 1e9, 0.0, 1e8),
}


@pytest.mark.parametrize("dt,floor", [(DT, 1e6), (1e3 * DT, 1.5e6)])
def test_edge_cases(dev, imported64, spec64, dt, floor):
    gt, stored = imported64
    arr = np.array(list(EDGE.values()), dtype=np.float64).T
    cells = dict(zip(W.FIELDS, arr))
    out = to_np(R.cool_step(gt, to_dev(cells, dev), dt, R.default_opts(T_floor=floor)))
    ref = S.step_be(S.TableSet(spec64, stored), *arr, dt, T_floor=floor)
    assert np.array_equal(out["status"], ref["status"])
    ok = (ref["status"] & R.ST_INVALID) == 0
    assert np.all(np.isnan(out["T_e_new"][~ok])) and np.all(np.isnan(out["Q_rad"][~ok]))
    for k in ("T_e_new", "T_i_new"):
        assert np.max(rel_err(out[k][ok], ref[k][ok])) < ENERGY_TOL, k


@pytest.mark.parametrize("n", [1, 63, 257, 4097])
def test_ragged_sizes(dev, imported64, cells0, be_ref0, n):
    gt, _ = imported64
    idx = np.arange(n) * 7 % 32768
    out = to_np(R.cool_step(gt, to_dev(cells0, dev, idx), DT))
    for k in ("T_e_new", "T_i_new"):
        assert np.max(rel_err(out[k], be_ref0[k][idx])) < ENERGY_TOL


def test_empty_input_is_a_noop(dev, imported64):
    gt, _ = imported64
    z = {k: torch.empty(0, dtype=torch.float64, device=dev) for k in W.FIELDS}
    out = R.cool_step(gt, z, DT)
    assert out["T_e_new"].numel() == 0


def test_bad_arguments_raise(dev, imported64, cells0):
    gt, _ = imported64
    st = to_dev(cells0, dev, np.arange(16))
    with pytest.raises(R.RadcoolError):
        R.cool_step(gt, st, -1.0)
    with pytest.raises(R.RadcoolError):
        R.cool_step(gt, st, DT, R.default_opts(variant="direct"))      # direct is rates-only
    with pytest.raises(R.RadcoolError):
        R.cool_step(gt, st, DT, R.default_opts(block=100))


def test_sizes_beyond_one_launch_are_refused(dev, imported64, cells0):
    """A cell count whose grid exceeds one launch is refused on the host
    (RC_EINVAL) before anything is launched or allocated, for the step in
    every scheme and for the adjoint; the tensors behind the pointers hold 16
    cells, so a launch would read far out of bounds (none happens)."""
    import ctypes
    gt, _ = imported64
    st = to_dev(cells0, dev, np.arange(16))
    out = R.cool_step(gt, st, DT)
    L = R.lib()
    s = R._state(st)
    o = R._out_struct(out)
    huge = 1 << 40
    for kw in (dict(), dict(scheme="rates"), dict(scheme="explicit16"), dict(passes=2), dict(variant="global")):
        opts = R.default_opts(**kw)
        assert L.rc_cool_step(gt.handle, ctypes.byref(s), huge, DT, ctypes.byref(opts), ctypes.byref(o), None) == -1
        assert b"too large" in L.rc_last_error(), kw
    fwd = R.Fwd(out["T_e_new"].data_ptr(), out["T_i_new"].data_ptr(), out["status"].data_ptr())
    cot = R.Cotangent(out["T_e_new"].data_ptr(), None, None, None)
    g = R.Grad(*[out["T_e_new"].data_ptr()] * 5, None)
    assert L.rc_cool_step_backward(gt.handle, ctypes.byref(s), huge, DT, ctypes.byref(R.default_opts()),
                                   ctypes.byref(fwd), ctypes.byref(cot), ctypes.byref(g), None) == -1
    assert b"too large" in L.rc_last_error()
    torch.cuda.synchronize()
    # the library still works
    again = R.cool_step(gt, st, DT)
    assert torch.equal(again["T_e_new"], out["T_e_new"])


def test_deterministic(dev, imported64, cells0):
    gt, _ = imported64
    st = to_dev(cells0, dev)
    a = R.cool_step(gt, st, DT)
    b = R.cool_step(gt, st, DT)
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_save_load_roundtrip(dev, gpu_tables64, cells0):
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "t.rct")
        gpu_tables64.save(path)
        back = R.Tables.load(path)
        r0, c0 = gpu_tables64.export()
        r1, c1 = back.export()
        assert np.array_equal(r0, r1) and np.array_equal(c0, c1)
        st = to_dev(cells0, dev, np.arange(4096))
        a = R.cool_step(gpu_tables64, st, DT)
        b = R.cool_step(back, st, DT)
        assert torch.equal(a["T_e_new"], b["T_e_new"]) and torch.equal(a["T_i_new"], b["T_i_new"])


# ------------------------------------------------------------------ full size, bench launch shape


def test_full_size_iid256_sampled(dev, oracle128):
    """256^3 cells, 128^3 tables, the launch configuration bench.py times.
    Sampled cells against the oracle; conservation at every cell."""
    ospec, otab = oracle128
    cells = W.workload(1)
    n = cells["n_e"].size
    st = to_dev(cells, dev)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(n, size=1024, replace=False))
    # rates tier: GPU-built tables vs oracle FP64 tables
    gbuilt = R.Tables.build(R.default_spec(128))
    rates = R.cool_step(gbuilt, st, DT, R.default_opts(scheme="rates"))
    ref_r = S.table_rates(S.TableSet(ospec, otab), *[cells[f][idx] for f in W.FIELDS])
    for g, r in (("Q_rad", "q_rad"), ("Q_cc", "q_cc")):
        assert np.max(rel_err(rates[g].cpu().numpy()[idx], ref_r[r])) < RATE_TOL, g
    del rates
    # energy tier on identical tables
    resid, coeffs, stored = storage_of(otab)
    gt = R.Tables.from_storage(R.default_spec(128), resid, coeffs)
    out = R.cool_step(gt, st, DT)
    ref = S.step_be(S.TableSet(ospec, stored), *[cells[f][idx] for f in W.FIELDS], DT)
    for k in ("T_e_new", "T_i_new"):
        assert np.max(rel_err(out[k].cpu().numpy()[idx], ref[k])) < ENERGY_TOL, k
    # every cell: finite, and the energy radiated equals dt Q_rad at the new state
    te, ti = out["T_e_new"], out["T_i_new"]
    assert bool(torch.isfinite(te).all()) and bool(torch.isfinite(ti).all())
    new_state = dict(st)
    new_state["T_e"], new_state["T_i"] = te, ti
    q_new = R.cool_step(gt, new_state, DT, R.default_opts(scheme="rates"))["Q_rad"]
    c = 1.5 * st["n_e"] * 1.380649e-16
    lost = c * ((st["T_e"] - te) + (st["T_i"] - ti))
    floor = (out["status"] & R.ST_FLOOR) != 0
    resid_e = (lost - DT * q_new).abs() / (c * (st["T_e"] + st["T_i"]))
    assert float(resid_e[~floor].max()) < 1e-9
    assert int((out["status"] & R.ST_MAXITER).sum()) == 0


@pytest.mark.parametrize("n,dt_scale", [(100_003, 1.0), (100_003, 1e3), (1, 1.0), (63, 1e3), (65, 1e3),
                                         (4099, 1e3)])
def test_newton_launch_shapes_agree(dev, imported64, n, dt_scale):
    """The default launch (64-thread workgroups) and 256-thread workgroups run
    the same per-cell steps; multiply-adds may be fused differently in the two
    builds, so values agree to rounding.  Ragged sizes leave partial
    workgroups; the stiff step (dt x 1e3) runs long Newton iterations."""
    gt, _ = imported64
    cells = W.workload(3, n=n)
    st = to_dev(cells, dev)
    dt = DT * dt_scale
    a = {k: v.cpu().numpy() for k, v in R.cool_step(gt, st, dt, R.default_opts(), diagnostics=True).items()}
    b = {k: v.cpu().numpy() for k, v in R.cool_step(gt, st, dt, R.default_opts(block=256),
                                                     diagnostics=True).items()}
    assert np.array_equal(a["status"], b["status"])
    for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "Q_brem", "Q_syn", "eta"):
        assert np.max(rel_err(a[k], b[k])) < 1e-12, k


@pytest.mark.parametrize("block", [0, 256])
def test_gas_floor_energy_tier(dev, imported64, spec64, block):
    """Per-cell gas-temperature floor: cells below it take the step with
    radiative cooling off (status 32), with one-wavefront and 256-thread
    workgroups."""
    from oracle import upstream as U
    gt, stored = imported64
    cells = W.workload(0)
    arr = [cells[f] for f in W.FIELDS]
    floor = np.median(arr[1] + arr[2]) * np.ones_like(arr[0])
    dt = 1e3 * DT
    st = to_dev(cells, dev)
    st["T_floor_gas"] = torch.from_numpy(floor).to(dev)
    out = to_np(R.cool_step(gt, st, dt, R.default_opts(block=block)))
    ref = U.step_with_gas_floor(S.TableSet(spec64, stored), *arr, dt, floor)
    assert np.array_equal(out["status"], ref["status"])
    off = (out["status"] & R.ST_GAS_FLOOR) != 0
    assert 0.3 < off.mean() < 0.7 and np.all(out["Q_rad"][off] == 0.0)
    for k in ("T_e_new", "T_i_new"):
        assert np.max(rel_err(out[k], ref[k])) < ENERGY_TOL, k


@pytest.mark.parametrize("n,dt_scale,floor", [(1, 1.0, 1e6), (4095, 1e3, 1e6), (4097, 1.0, 1e6),
                                               (100_003, 1.0, 1e6), (100_003, 1e3, 3e7), (65_537, 1e2, 5e7)])
def test_two_pass_equals_one_pass(dev, imported64, n, dt_scale, floor):
    """The two-pass Newton step (first round in cell order, per-tile sort by
    the first step, resumed rounds) runs the single pass's per-cell steps;
    the two are separate kernels, so multiply-adds may be fused differently:
    values agree to rounding, status exactly.  Sizes cover one cell, both
    sides of a 4096-cell tile boundary and many tiles; the stiff steps and the
    raised floors make first rounds end in floor probes."""
    gt, _ = imported64
    cells = W.workload(3, n=n)
    st = to_dev(cells, dev)
    dt = DT * dt_scale
    one = to_np(R.cool_step(gt, st, dt, R.default_opts(T_floor=floor, passes=1), diagnostics=True))
    two = to_np(R.cool_step(gt, st, dt, R.default_opts(T_floor=floor, passes=2), diagnostics=True))
    assert np.array_equal(one["status"], two["status"])
    for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "Q_brem", "Q_syn", "eta"):
        assert np.max(rel_err(one[k], two[k])) < 1e-12, k
    if floor > 1e6:
        assert int(np.sum(one["status"] & R.ST_FLOOR)) > 0
