"""GPU parity of the upstream inputs (thermal scale height, gas-temperature
floor) and of the radiation-pressure temperature correction against the
oracle (FP64 on both sides; 1e-13 relative allows for fused multiply-adds)."""
import numpy as np
import pytest

from conftest import rel_err
from oracle import upstream as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2505_08855_amd.radcool")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return torch.device("cuda:0")


@pytest.mark.parametrize("n", [1, 1000, 1_000_003])
def test_disk_inputs_match_oracle(dev, n):
    rng = np.random.default_rng(n)
    rho = 10 ** rng.uniform(-14, -2, n)
    P = 10 ** rng.uniform(-6, 0.5, n) * rho * 2.99792458e10 ** 2
    u = 1.5 * P
    r = 10 ** rng.uniform(0.2, 3, n)
    if n > 1:
        rho[0] = np.nan                       # an invalid cell
    prm = R.disk_params()
    t = lambda a: torch.from_numpy(a).to(dev)
    out = R.disk_inputs({"rho": t(rho), "P": t(P), "u": t(u), "r": t(r)}, prm)
    H, Tf = out["H_th"].cpu().numpy(), out["T_floor_gas"].cpu().numpy()
    ok = np.isfinite(rho)
    assert np.all(np.isnan(H[~ok])) and np.all(np.isnan(Tf[~ok]))
    assert np.max(rel_err(H[ok], U.scale_height(rho[ok], P[ok], u[ok], r[ok], prm.spin, prm.gamma, prm.r_g))) < 1e-13
    assert np.max(rel_err(Tf[ok], U.floor_temperature(r[ok], prm.spin, prm.h_floor))) < 1e-13


@pytest.mark.parametrize("n", [1, 4097, 1_000_003])
def test_rad_pressure_correction_matches_oracle(dev, n):
    rng = np.random.default_rng(n + 7)
    n_e = 10 ** rng.uniform(14, 24, n)
    T_e = 10 ** rng.uniform(5, 10, n)
    H = 10 ** rng.uniform(5, 9, n)
    t = lambda a: torch.from_numpy(a).to(dev)
    T, thick = R.rad_pressure_correction(t(n_e), t(T_e), t(H))
    T, thick = T.cpu().numpy(), thick.cpu().numpy().astype(bool)
    ref, rthick = U.rad_pressure_temperature(n_e, T_e, T_e, H)
    assert np.array_equal(thick, rthick)
    assert np.max(rel_err(T, ref)) < 1e-13
    assert np.array_equal(T[~thick], T_e[~thick])


def _coupling_case(n, seed):
    rng = np.random.default_rng(seed)
    ne = 10 ** rng.uniform(10, 20, n)
    te = 10 ** rng.uniform(7, 11, n)
    ti = te * 10 ** rng.uniform(0, 2, n)
    ten = te * (1 - rng.uniform(-0.5, 0.5, n))
    tin = ti * (1 - rng.uniform(-0.01, 0.01, n))
    v = rng.uniform(-0.5, 0.5, (n, 3))
    g = 1.0 / np.sqrt(1.0 - (v ** 2).sum(1))
    u = [-g] + [g * v[:, k] for k in range(3)]
    U0 = [rng.normal(size=n) * 1e3 for _ in range(4)]
    sg = rng.uniform(0.5, 2.0, n)
    return ne, te, ti, ten, tin, u, U0, sg


@pytest.mark.parametrize("n", [1, 1000, 1_000_003])
def test_apply_cooling_matches_oracle(dev, n):
    """Downstream coupling in place on the device against the oracle; an
    invalid step keeps U and reports lambda = NaN."""
    ne, te, ti, ten, tin, u, U0, sg = _coupling_case(n, n + 7)
    if n > 1:
        tin[n // 2] = np.nan
    dt = 4.9e-8
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    Ud = [t(a) for a in U0]
    lam = R.apply_cooling({"n_e": t(ne), "T_e": t(te), "T_i": t(ti)}, {"T_e_new": t(ten), "T_i_new": t(tin)},
                          [t(a) for a in u], Ud, dt, sqrt_g=t(sg)).cpu().numpy()
    ref_l = U.cooling_lambda(ne, te, ti, ten, tin, dt)
    ref_U = U.apply_cooling(U0, u, ref_l, dt, sqrt_g=sg)
    ok = np.isfinite(ref_l)
    assert np.array_equal(np.isfinite(lam), ok)
    assert np.max(rel_err(lam[ok], ref_l[ok])) < 1e-13
    for mu in range(4):
        got = Ud[mu].cpu().numpy()
        # U + f u with a fused multiply-add on the device: rounding is relative
        # to the terms, not to their (possibly cancelling) sum
        scale = np.abs(U0[mu]) + np.abs(np.where(ok, dt * sg * ref_l * u[mu], 0.0))
        assert np.max(np.abs(got - ref_U[mu]) / scale) < 1e-14
        assert np.array_equal(got[~ok], U0[mu][~ok])


def test_apply_cooling_of_a_newton_step(dev):
    """The GPU Newton step followed by the coupling in the fluid frame: U_0
    gains dt lambda, and lambda equals Q_rad at the step's new temperatures
    (the energy balance of backward Euler, to the energy tier)."""
    from paper_2505_08855_amd import workloads as W
    gt = R.Tables.build(R.default_spec(64))
    cells = W.workload(0, n=20_000)
    st = {k: torch.from_numpy(cells[k]).to(dev) for k in W.FIELDS}
    dt = W.DT_DEFAULT * 1e2
    out = R.cool_step(gt, st, dt, R.default_opts())
    n = cells["n_e"].size
    z = torch.zeros(n, dtype=torch.float64, device=dev)
    u = [-torch.ones(n, dtype=torch.float64, device=dev), z, z, z]
    U0 = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(4)]
    lam = R.apply_cooling(st, out, u, U0, dt)
    new = dict(st)
    new["T_e"], new["T_i"] = out["T_e_new"], out["T_i_new"]
    q_new = R.cool_step(gt, new, dt, R.default_opts(scheme="rates"))["Q_rad"].cpu().numpy()
    lam, U00 = lam.cpu().numpy(), U0[0].cpu().numpy()
    assert np.max(rel_err(U00, dt * lam)) < 1e-15
    assert all(float(U0[mu].abs().max()) == 0.0 for mu in (1, 2, 3))
    keep = (out["status"].cpu().numpy() & R.ST_FLOOR) == 0
    u_gas = 1.5 * cells["n_e"] * 1.380649e-16 * (cells["T_e"] + cells["T_i"])
    assert keep.sum() > 0.9 * n
    assert np.max(np.abs(lam - q_new)[keep] * dt / u_gas[keep]) < 1e-9
    gt.destroy()
