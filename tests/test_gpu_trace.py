"""Per-stage timing inside the library (mls_context_trace): the stages of
each kind of call, positive times that add up to the record's total, the
contraction form, and one JSON line per call in the trace file."""
import json
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_stage_times_and_json_lines(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_0677_amd import api, workloads as wl
    note("case trace")
    ctx = api.Context(0)
    path = tmp_path / "trace.jsonl"
    ctx.trace(True, str(path))
    w = wl.c2(grid_side=256, n=2000)
    P = torch.from_numpy(w.points).cuda()
    V = torch.from_numpy(w.values).cuda()
    F, _ = api.fit(P, V, w.grid, basis="linear", h=0.03, ctx=ctx)
    rec = ctx.trace_last()
    assert rec["call"] == "fit" and rec["form"] == 0 and list(rec["stages"]) == ["contract"]
    api.fit(P, V, w.grid, basis="quadratic", h=0.06, precision="bf16", ctx=ctx, lp_form=2)
    rec = ctx.trace_last()
    assert rec["form"] == 2 and list(rec["stages"]) == ["stage", "contract"]
    api.fit(P, V, w.grid, basis="quadratic", h=0.06, precision="bf16", ctx=ctx, lp_form=1)
    assert ctx.trace_last()["form"] == 1
    api.fit(P, V, w.grid, basis="quadratic", weight="wendland", h=0.1, precision="bf16",
            ctx=ctx)
    rec = ctx.trace_last()
    assert list(rec["stages"]) == ["stage", "cells", "contract"]
    for v in rec["stages"].values():
        assert v > 0.0
    assert abs(sum(rec["stages"].values()) - rec["total_ms"]) < 1e-9
    iso = torch.from_numpy(w.iso()).cuda()
    api.contour(F, w.grid, iso, ctx=ctx)
    assert ctx.trace_last()["call"] == "contour"
    ctx.trace(False)
    # calls after tracing is off add no line
    api.fit(P, V, w.grid, basis="linear", h=0.03, ctx=ctx)
    torch.cuda.synchronize()
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    # the contour's retry on capacity traces both of its calls
    assert [x["call"] for x in lines[:4]] == ["fit"] * 4
    assert all(x["call"] == "contour" for x in lines[4:]) and len(lines) >= 5
    assert lines[0]["n"] == 2000 and lines[0]["d"] == 13 and lines[0]["width"] == 256
    assert lines[1]["form"] == 2
    for x in lines:
        assert x["total_ms"] > 0.0
        assert abs(sum(x["stages_ms"].values()) - x["total_ms"]) < 1e-6
    ctx.close()
