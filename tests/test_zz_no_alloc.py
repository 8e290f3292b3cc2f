"""The allocation-free step entry point, rc_cool_step_noalloc, against
rc_cool_step through the C ABI.

Same kernels, so the results are the same bits when both read the same table
layout; a fresh table handle has no cell-blocked copy yet, and then the
allocation-free call reads the node layout, whose results agree with the
cell-blocked ones to rounding (1e-12, identical status).  Two calls in a row,
the second smaller, so that the second reads a static scratch still holding
the first call's contents; the size limit and the missing copy are refused
on the host.
"""
import numpy as np
import pytest

from conftest import rel_err
from paper_2505_08855_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2505_08855_amd.radcool")
DT = W.DT_DEFAULT
KEYS = ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "status")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return torch.device("cuda:0")


def state_of(cells, dev, n):
    return {k: torch.from_numpy(np.ascontiguousarray(cells[k][:n])).to(dev) for k in W.FIELDS}


def empty_out(n, dev):
    out = {k: torch.full((n,), float("nan"), dtype=torch.float64, device=dev) for k in KEYS[:4]}
    out["status"] = torch.full((n,), 0xEE, dtype=torch.uint8, device=dev)
    return out


def check_same(a, b, exact):
    assert torch.equal(a["status"], b["status"])
    for k in KEYS[:4]:
        if exact:
            assert torch.equal(a[k], b[k]), k
        else:
            err = np.max(rel_err(a[k].cpu().numpy(), b[k].cpu().numpy()))
            assert err < 1e-12, (k, err)


def test_noalloc_matches_cool_step_twice(dev):
    cells = W.workload(1, n=R.NOALLOC_MAX_CELLS)
    big, small = R.NOALLOC_MAX_CELLS, 4099
    tables = R.Tables.build(R.default_spec(64))
    opts = R.default_opts(passes=2)          # the two-pass step: its scratch is the static array
    print("noalloc: fresh tables, %d cells, then %d cells" % (big, small), flush=True)

    # fresh handle: no cell-blocked copy, so the call reads the node layout
    st = state_of(cells, dev, big)
    a = R.cool_step_noalloc(tables, st, DT, empty_out(big, dev), opts)
    ref_global = R.cool_step(tables, st, DT, R.default_opts(variant="global", passes=2))
    torch.cuda.synchronize()
    check_same(a, ref_global, exact=True)
    # the explicit cell-blocked variant needs the copy, which this entry point never builds
    with pytest.raises(R.RadcoolError) as e:
        R.cool_step_noalloc(tables, st, DT, empty_out(big, dev), R.default_opts(variant="cell", passes=2))
    assert e.value.code == -5

    # rc_cool_step builds the copy; both entry points then read it
    ref = R.cool_step(tables, st, DT, opts)
    b = R.cool_step_noalloc(tables, st, DT, empty_out(big, dev), opts)
    torch.cuda.synchronize()
    check_same(b, ref, exact=True)
    check_same(b, ref_global, exact=False)

    # second call, smaller, on other cells: the scratch still holds the first call's records
    st2 = {k: v[-small:].contiguous() for k, v in state_of(cells, dev, big).items()}
    c = R.cool_step_noalloc(tables, st2, DT, empty_out(small, dev), opts)
    ref2 = R.cool_step(tables, st2, DT, opts)
    torch.cuda.synchronize()
    check_same(c, ref2, exact=True)

    # every scheme and the one-pass form go through it too
    for kw in (dict(), dict(passes=1), dict(scheme="rates"), dict(scheme="explicit16")):
        o = R.default_opts(**kw)
        x = R.cool_step_noalloc(tables, st2, DT, empty_out(small, dev), o)
        y = R.cool_step(tables, st2, DT, o)
        torch.cuda.synchronize()
        check_same(x, y, exact=True)
    tables.destroy()


def test_noalloc_size_limit(dev):
    tables = R.Tables.build(R.default_spec(16))
    n = R.NOALLOC_MAX_CELLS + 1
    st = {k: torch.ones(n, dtype=torch.float64, device=dev) for k in W.FIELDS}
    with pytest.raises(R.RadcoolError) as e:
        R.cool_step_noalloc(tables, st, DT, empty_out(n, dev))
    assert e.value.code == -1 and b"RC_NOALLOC_MAX_CELLS" in R.lib().rc_last_error()
    # n = 0 is a no-op
    st0 = {k: v[:0] for k, v in st.items()}
    R.cool_step_noalloc(tables, st0, DT, empty_out(0, dev))
    tables.destroy()
