"""The batched form at full size: 4096 uneven AMR blocks x 8 accretion states
(about 126 M cell-updates, 32,768 work items) through one captured persistent
launch on a fixed grid of one workgroup per compute unit, so that every
workgroup walks the work queue for many items (counted by the kernel).

Checked against the plain step run state by state on every cell (same
per-cell code: 1e-12 and identical status) and against the oracle's backward
Euler on identical table data (the oracle's 64^3 tables imported in storage
form) on cells sampled from every state (1e-9)."""
import numpy as np
import pytest

from conftest import rel_err
from oracle import step as S
from oracle import tables as T
from paper_2505_08855_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2505_08855_amd.radcool")
N_STATES = 8


@pytest.fixture(scope="module")
def full(spec64, tables64):
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    dev = torch.device("cuda:0")
    print("generating 4096 blocks x 8 states", flush=True)
    cells, blocks, _ = W.amr_blocks()
    dts = W.DT_DEFAULT * (1.0 + 0.25 * np.arange(N_STATES))       # a different dt per state
    co, re, st = T.quantize_tables(tables64)
    resid = np.concatenate([re[k].ravel() for k in T.TABLE_NAMES])
    coeffs = np.stack([co[k] for k in T.TABLE_NAMES])
    gt = R.Tables.from_storage(R.default_spec(64), resid, coeffs)
    state = {k: torch.from_numpy(cells[k]).to(dev) for k in W.FIELDS}
    bdev, nb = R.blocks_to_device(blocks, dev)
    return {"dev": dev, "cells": cells, "blocks": blocks, "dts": dts, "tables": gt,
            "ts": S.TableSet(T.TableSpec.default(64), st), "state": state, "bdev": bdev, "nb": nb}


def test_full_size_plan_on_one_workgroup_per_cu(full):
    dev = full["dev"]
    n = full["cells"]["n_e"].size
    assert n > 120_000_000 and full["nb"] == 4096 * N_STATES
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    plan = R.Plan(full["tables"], full["state"], full["bdev"], full["nb"], full["dts"], R.default_opts(grid=cus),
                  autotune=False)
    assert plan.info()["grid"] == cus
    plan.launch()
    items = plan.workgroup_items()
    print("items per workgroup: min %d, median %d, max %d" % (items.min(), np.median(items), items.max()), flush=True)
    assert items.size == cus and int(items.sum()) == full["nb"]
    assert items.min() >= 2
    out = plan.out

    # the plain step, state by state (a state's cells are contiguous)
    blocks = full["blocks"]
    for s in range(N_STATES):
        lo = min(b[0] for b in blocks if b[2] == s)
        hi = max(b[0] + b[1] for b in blocks if b[2] == s)
        sub = {k: v[lo:hi] for k, v in full["state"].items()}
        ref = R.cool_step(full["tables"], sub, full["dts"][s])
        assert torch.equal(out["status"][lo:hi], ref["status"]), s
        for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc"):
            a, b = out[k][lo:hi], ref[k]
            err = ((a - b).abs() / b.abs().clamp_min(1e-300)).max().item()
            assert err < 1e-12, (s, k, err)
        del ref
    torch.cuda.synchronize()

    # the oracle on identical table data, cells from every state
    rng = np.random.default_rng(44)
    cells = full["cells"]
    host = {k: out[k].cpu().numpy() for k in ("T_e_new", "T_i_new")}
    for s in range(N_STATES):
        blks = [blocks[j] for j in rng.choice([j for j, b in enumerate(blocks) if b[2] == s], 16, replace=False)]
        idx = np.concatenate([b[0] + rng.choice(b[1], 4, replace=False) for b in blks])
        ref = S.step_be(full["ts"], *[cells[f][idx] for f in W.FIELDS], full["dts"][s])
        for k in ("T_e_new", "T_i_new"):
            assert np.max(rel_err(host[k][idx], ref[k])) < 1e-9, (s, k)
    plan.destroy()
