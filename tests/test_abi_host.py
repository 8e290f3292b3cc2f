"""The C-ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before anything is launched.  CPU only: no call here
launches a kernel."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

R = pytest.importorskip("paper_2505_08855_amd.radcool")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(R.LIB_PATH):
        pytest.fail("libradcool.so is not built (python -m paper_2505_08855_amd.build)")
    return R.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "radcool.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(rc_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(R.EXPORTED)


def test_constants_match_oracle(L):
    from oracle import constants as K
    lib_c = R.constants()
    want = [K.C_LIGHT, K.K_B, K.H_PLANCK, K.M_E, K.M_P, K.E_CHARGE, K.SIGMA_T, K.SIGMA_SB]
    assert lib_c == want


def test_default_spec_and_opts(L):
    s = R.default_spec(64)
    assert list(s.cool.n) == [64, 64, 64] and list(s.coul.n) == [64, 64, 64]
    assert list(s.cool.lo) == [15.0, 5.95, -0.5] and list(s.cool.hi) == [29.0, 12.05, 10.5]
    assert list(s.coul.lo) == [9.5, 5.95, 5.95] and list(s.coul.hi) == [20.5, 12.05, 14.05]
    assert s.ln_lambda == 20.0
    # the oracle's default axes are the same numbers
    from oracle import tables as T
    o = T.TableSpec.default(64)
    for a in range(3):
        assert (o.cool[a].lo, o.cool[a].hi) == (s.cool.lo[a], s.cool.hi[a])
        assert (o.coul[a].lo, o.coul[a].hi) == (s.coul.lo[a], s.coul.hi[a])
    op = R.default_opts()
    assert (op.scheme, op.variant, op.max_iter, op.block, op.T_floor, op.tol) == (0, 0, 60, 0, 1e6, 1e-12)


def test_argument_errors_without_launch(L):
    assert L.rc_default_spec(None, 64) == -1
    s = R.TableSpec()
    assert L.rc_default_spec(ctypes.byref(s), 1) == -1
    assert L.rc_default_opts(None) == -1
    # invalid spec is rejected before any device work
    bad = R.default_spec(64)
    bad.cool.hi[0] = bad.cool.lo[0]
    h = ctypes.c_void_p()
    assert L.rc_build_tables(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    assert not h.value
    assert b"spec" in L.rc_last_error()
    assert L.rc_build_tables(ctypes.byref(bad), None, None) == -1
    # import with NULL data
    good = R.default_spec(8)
    assert L.rc_tables_import(ctypes.byref(good), None, None, None, ctypes.byref(h)) == -1
    # step with a NULL / bogus handle
    st = R.State()
    o = R.Out()
    op = R.default_opts()
    assert L.rc_cool_step(None, ctypes.byref(st), 10, 1e-8, ctypes.byref(op), ctypes.byref(o), None) == -5
    fake = (ctypes.c_uint32 * 64)()
    assert L.rc_cool_step(ctypes.cast(fake, ctypes.c_void_p), ctypes.byref(st), 10, 1e-8, ctypes.byref(op),
                          ctypes.byref(o), None) == -5
    assert L.rc_tables_destroy(ctypes.cast(fake, ctypes.c_void_p)) == -5
    assert L.rc_tables_destroy(None) == 0
    assert L.rc_tables_export(None, None, None) == -5
    assert L.rc_tables_save(None, b"/tmp/x") == -5
    assert L.rc_tables_load(None, None, ctypes.byref(h)) == -1
    assert L.rc_tables_load(b"/nonexistent/file.rct", None, ctypes.byref(h)) == -6


def test_tables_load_rejects_corrupt_files(L, tmp_path):
    h = ctypes.c_void_p()
    p = tmp_path / "junk.rct"
    p.write_bytes(b"RCTABLE1" + b"\0" * 64)
    assert L.rc_tables_load(str(p).encode(), None, ctypes.byref(h)) == -6
    p.write_bytes(b"NOTMAGIC" + b"\0" * 400)
    assert L.rc_tables_load(str(p).encode(), None, ctypes.byref(h)) == -6


def test_selftest_argument_checks(L):
    s = R.default_spec(8)
    v = ctypes.c_double()
    assert L.rc_selftest_node_host(ctypes.byref(s), 4, 0, 0, 0, ctypes.byref(v)) == -1
    assert L.rc_selftest_node_host(ctypes.byref(s), 0, 8, 0, 0, ctypes.byref(v)) == -1
    assert L.rc_selftest_special_host(10, None, None, 1) == -1
    op = R.default_opts(max_iter=0)
    x = np.ones(1)
    resid = np.zeros(4 * 512, dtype=np.float32)
    co = np.zeros(16)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    for bad_dt in (0.0, -1.0, float("nan"), float("inf")):
        assert L.rc_selftest_step_host(ctypes.byref(s), P(resid), P(co), *[P(x)] * 5, None, 1, bad_dt,
                                       ctypes.byref(R.default_opts()), None, None, None, None, None) == -1
    assert L.rc_selftest_step_host(ctypes.byref(s), P(resid), P(co), *[P(x)] * 5, None, 1, 1e-8,
                                   ctypes.byref(op), None, None, None, None, None) == -1
    for field, val in (("scheme", 7), ("variant", 9), ("T_floor", -1.0), ("tol", 0.0), ("block", 96),
                       ("rate_dtype", 2), ("reserved", 1), ("grid", -1), ("grid", 65537), ("passes", 3)):
        op = R.default_opts(**{field: val})
        assert L.rc_selftest_step_host(ctypes.byref(s), P(resid), P(co), *[P(x)] * 5, None, 1, 1e-8,
                                       ctypes.byref(op), None, None, None, None, None) == -1, field


def test_reading_switches_are_checked(L):
    """Spec fields outside their enums are rejected; tables of the literal
    Compton exponent refuse every scheme but the rates."""
    h = ctypes.c_void_p()
    for field, val in (("compton_exponent", 2), ("theta_i_mass", -1), ("reserved", 3), ("value_dtype", 5)):
        bad = R.default_spec(8)
        setattr(bad, field, val)
        assert L.rc_build_tables(ctypes.byref(bad), None, ctypes.byref(h)) == -1, field
        assert not h.value
    lit = R.default_spec(8, compton="literal")
    x = np.ones(1)
    resid = np.zeros(4 * 512, dtype=np.float32)
    co = np.zeros(16)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    for scheme in ("newton", "explicit16"):
        assert L.rc_selftest_step_host(ctypes.byref(lit), P(resid), P(co), *[P(x)] * 5, None, 1, 1e-8,
                                       ctypes.byref(R.default_opts(scheme=scheme)), None, None, None, None,
                                       None) == -4, scheme
    assert b"literal Compton" in L.rc_last_error()


LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "radcool.h"
#define S(T) printf(#T " size %zu\n", sizeof(T))
#define O(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))
int main(void) {
  S(rc_axes); S(rc_table_spec); S(rc_state); S(rc_out); S(rc_step_opts); S(rc_block); S(rc_fwd);
  S(rc_cotangent); S(rc_grad); S(rc_disk_params); S(rc_coupling); S(rc_axes4);
  O(rc_table_spec, ln_lambda); O(rc_table_spec, value_dtype); O(rc_table_spec, compton_exponent);
  O(rc_table_spec, theta_i_mass); O(rc_table_spec, reserved); O(rc_table_spec, external_storage);
  O(rc_table_spec, external_bytes);
  O(rc_step_opts, T_floor); O(rc_step_opts, tol); O(rc_step_opts, passes); O(rc_step_opts, grid);
  O(rc_step_opts, rate_dtype); O(rc_step_opts, reserved);
  O(rc_out, Q_rad); O(rc_out, status); O(rc_out, eta);
  O(rc_block, n_cells); O(rc_block, state_id);
  return 0;
}
"""


def test_struct_layouts_match_the_binding(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes
    and field offsets (gcc, the header compiled as C)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    types = {"rc_axes": R.Axes, "rc_table_spec": R.TableSpec, "rc_state": R.State, "rc_out": R.Out,
             "rc_step_opts": R.StepOpts, "rc_block": R.Block, "rc_fwd": R.Fwd, "rc_cotangent": R.Cotangent,
             "rc_grad": R.Grad, "rc_disk_params": R.DiskParams, "rc_coupling": R.Coupling, "rc_axes4": R.Axes4}
    seen = 0
    for ln in lines:
        parts = ln.split()
        if len(parts) == 3 and parts[1] == "size":
            assert ctypes.sizeof(types[parts[0]]) == int(parts[2]), parts[0]
            seen += 1
        elif len(parts) == 3:
            assert getattr(types[parts[0]], parts[1]).offset == int(parts[2]), (parts[0], parts[1])
            seen += 1
    assert seen == 12 + 18


def test_apply_cooling_rejects_bad_arguments(L):
    """Host-side argument checks of rc_apply_cooling (nothing is launched)."""
    c = R.Coupling()
    one = np.ones(4)
    p = one.ctypes.data_as(ctypes.c_void_p).value
    for mu in range(4):
        c.u_cov[mu] = p
    args = [p] * 5
    assert L.rc_apply_cooling(*args, -1, 1.0, ctypes.byref(c), None, None) == -1      # n < 0
    assert L.rc_apply_cooling(*args, 4, 0.0, ctypes.byref(c), None, None) == -1       # dt <= 0
    assert L.rc_apply_cooling(*args, 4, float("nan"), ctypes.byref(c), None, None) == -1
    assert L.rc_apply_cooling(*args, 4, 1.0, None, None, None) == -1                  # coupling NULL
    c.u_cov[2] = None
    assert L.rc_apply_cooling(*args, 4, 1.0, ctypes.byref(c), None, None) == -1       # velocity NULL
    assert L.rc_apply_cooling(*args, 0, 1.0, ctypes.byref(c), None, None) == 0        # empty: no-op


def test_variant_names_match_the_header():
    """The binding's variant names carry the header's enum values, and the
    library accepts each of them and rejects the next value (host check, no
    launch: the host self-test runs the per-cell code on the CPU)."""
    src = open(os.path.join(ROOT, "include", "radcool.h")).read()
    enum = dict((k.lower(), int(v)) for k, v in re.findall(r"RC_VARIANT_(\w+) = (\d+)", src))
    assert enum == R.VARIANTS
    s = R.default_spec(4)
    n = 4 * 4 * 4
    resid = np.zeros(4 * n, dtype=np.float32)
    co = np.zeros(16)
    x = np.ones(1)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    L = R.lib()
    for name, val in R.VARIANTS.items():
        if name == "direct":
            continue          # rates scheme only
        op = R.default_opts(variant=name)
        assert L.rc_selftest_step_host(ctypes.byref(s), P(resid), P(co), *[P(x)] * 5, None, 1, 1e-8,
                                       ctypes.byref(op), None, None, None, None, None) == 0, name
    op = R.default_opts()
    op.variant = max(R.VARIANTS.values()) + 1
    assert L.rc_selftest_step_host(ctypes.byref(s), P(resid), P(co), *[P(x)] * 5, None, 1, 1e-8,
                                   ctypes.byref(op), None, None, None, None, None) == -1


def _up(b):
    return (b + 255) // 256 * 256


@pytest.mark.parametrize("n,dtype", [((64, 64, 64), "f32"), ((128, 128, 128), "f32"), ((5, 7, 9), "f32"),
                                     ((64, 64, 64), "bf16"), ((5, 7, 9), "bf16")])
def test_storage_bytes_is_the_layout_of_the_parts(L, n, dtype):
    """rc_tables_storage_bytes: geometry record, node tables (16 / 4 bytes per
    cooling / Coulomb node in FP32, 8 / 2 in bfloat16) and, for FP32, the
    cell-blocked copy (64 / 32 bytes per table cell), each 256-byte aligned."""
    ax = [(m, 0.0, 1.0) for m in n]
    s = R.spec_from_axes(ax, ax[::-1], value_dtype=dtype)
    vc = vk = n[0] * n[1] * n[2]
    cells = (n[0] - 1) * (n[1] - 1) * (n[2] - 1)
    bf = dtype == "bf16"
    got = R.storage_bytes(s)
    parts = [_up((8 if bf else 16) * vc), _up((2 if bf else 4) * vk)]
    if not bf:
        parts += [_up(64 * cells), _up(32 * cells)]
    # the geometry record: one 256-byte-aligned slot ahead of the tables
    assert got - sum(parts) in (256, 512)
    assert got % 256 == 0
    # the external fields of the spec do not enter the size
    s.external_storage = 4096
    s.external_bytes = 1
    assert R.storage_bytes(s) == got


def test_storage_bytes_and_external_fields_are_checked(L):
    n = ctypes.c_uint64()
    assert L.rc_tables_storage_bytes(None, ctypes.byref(n)) == -1
    s = R.default_spec(8)
    assert L.rc_tables_storage_bytes(ctypes.byref(s), None) == -1
    bad = R.default_spec(8)
    bad.cool.n[0] = 1
    assert L.rc_tables_storage_bytes(ctypes.byref(bad), ctypes.byref(n)) == -1
    # a size without storage is an inconsistent spec: refused before any device call
    h = ctypes.c_void_p()
    s.external_bytes = 1 << 20
    assert L.rc_build_tables(ctypes.byref(s), None, ctypes.byref(h)) == -1
    assert not h.value
    resid = np.zeros(4 * 512, dtype=np.float32)
    co = np.zeros(16)
    assert L.rc_tables_import(ctypes.byref(s), resid.ctypes.data_as(ctypes.c_void_p),
                              co.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(h)) == -1
    d = R.default_spec(8)
    assert d.external_storage is None and d.external_bytes == 0
