"""Tables in caller-owned device memory (rc_table_spec.external_storage).

The tables built or imported into a caller's buffer are the same tables as
library-owned ones: every scheme gives bit-identical outputs on the same
inputs.  FP32 tables in external storage carry their cell-blocked copy from
the build on, so the allocation-free entry point can read it at once; the
library neither frees nor modifies the buffer on destroy; storage that is too
small, misaligned or not device memory is refused."""
import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def state(dev):
    cells = W.workload(0)
    return {k: torch.from_numpy(cells[k]).to(dev) for k in W.FIELDS}


def buffer(spec, dev, extra=0):
    return torch.zeros(R.storage_bytes(spec) + extra, dtype=torch.uint8, device=dev)


def outputs_equal(a, b):
    return all(torch.equal(a[k], b[k]) for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "status"))


@pytest.mark.parametrize("kw", [dict(), dict(scheme="rates"), dict(scheme="explicit16"), dict(variant="global"),
                                dict(variant="lds"), dict(passes=2)])
def test_built_into_external_storage_equals_library_owned(dev, state, kw):
    spec = R.default_spec(64)
    buf = buffer(spec, dev)
    ext = R.Tables.build(spec, storage=buf)
    own = R.Tables.build(spec)
    assert np.array_equal(ext.export()[0], own.export()[0])
    assert outputs_equal(R.cool_step(ext, state, DT, R.default_opts(**kw)),
                         R.cool_step(own, state, DT, R.default_opts(**kw)))
    ext.destroy()
    own.destroy()


def test_imported_tables_and_the_cell_copy_are_ready(dev, state):
    """Import into external storage: identical to a library-owned import, and
    the allocation-free step reads the cell-blocked copy without any earlier
    call having built it (a library-owned fresh table set refuses that)."""
    spec = R.default_spec(64)
    resid, coeffs = R.Tables.build(spec).export()
    buf = buffer(spec, dev)
    ext = R.Tables.from_storage(spec, resid, coeffs, storage=buf)
    own = R.Tables.from_storage(spec, resid, coeffs)
    n = state["n_e"].numel()

    def empty():
        o = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")}
        o["status"] = torch.empty(n, dtype=torch.uint8, device=dev)
        return o

    cell = R.default_opts(variant="cell")
    a = R.cool_step_noalloc(ext, state, DT, empty(), cell)
    with pytest.raises(R.RadcoolError):
        R.cool_step_noalloc(own, state, DT, empty(), cell)
    assert outputs_equal(a, R.cool_step(own, state, DT, cell))
    ext.destroy()
    own.destroy()


def test_destroy_leaves_the_buffer_to_the_caller(dev, state):
    spec = R.default_spec(32)
    buf = buffer(spec, dev)
    t = R.Tables.build(spec, storage=buf)
    before = buf.clone()
    assert int(before.count_nonzero()) > 0
    ref = R.cool_step(t, state, DT)
    t.destroy()
    torch.cuda.synchronize()
    assert torch.equal(buf, before)
    # a second table set in the same buffer after the first is gone
    t2 = R.Tables.build(spec, storage=buf)
    assert outputs_equal(R.cool_step(t2, state, DT), ref)
    t2.destroy()


def test_bfloat16_tables_in_external_storage(dev, state):
    """No cell-blocked copy for bfloat16 tables: a smaller buffer, node-layout reads."""
    spec = R.default_spec(64, value_dtype="bf16")
    assert R.storage_bytes(spec) < R.storage_bytes(R.default_spec(64)) // 8
    buf = buffer(spec, dev)
    ext = R.Tables.build(spec, storage=buf)
    own = R.Tables.build(spec)
    assert outputs_equal(R.cool_step(ext, state, DT), R.cool_step(own, state, DT))
    ext.destroy()
    own.destroy()


def test_unusable_storage_is_refused(dev):
    spec = R.default_spec(16)
    need = R.storage_bytes(spec)
    small = torch.zeros(need - 256, dtype=torch.uint8, device=dev)
    with pytest.raises(R.RadcoolError, match="external_bytes"):
        R.Tables.build(spec, storage=small)
    big = torch.zeros(need + 512, dtype=torch.uint8, device=dev)
    with pytest.raises(R.RadcoolError, match="aligned"):
        R.Tables.build(spec, storage=big[64:])
    host = torch.zeros(need, dtype=torch.uint8)
    with pytest.raises(R.RadcoolError, match="device memory"):
        R.Tables.build(spec, storage=host)
    # the library still works after the refusals
    t = R.Tables.build(spec, storage=big)
    t.destroy()
