"""Per-step records as JSON lines (MX_STATS): one line per step with the
same counts and norms mx_step returns."""
import json

import pytest

from paper_1907_13088_amd import inputs as I
from paper_1907_13088_amd import mx

from gpu_helpers import gpu_config, torch_fields

pytestmark = pytest.mark.gpu


def test_stats_json_lines(tmp_path, monkeypatch):
    import torch
    path = tmp_path / "steps.jsonl"
    monkeypatch.setenv("MX_STATS", str(path))
    w = I.modes_2d((200, 136), nmodes=24, npulses=4, filter_passes=2, m=200, steps=5, seed=4301, dtype="f64")
    g = mx.Grid(gpu_config(w, tol=1e-10))
    g.bind(torch_fields(w.E, "f64"), torch_fields(w.B, "f64"))
    g.set_current(torch_fields(w.J0, "f64"))
    st = g.step(3, env=list(w.env[:3]), stats=True)
    st += g.step(2, env=list(w.env[3:5]), stats=False) or []
    torch.cuda.synchronize()
    g.close()
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [x["step"] for x in lines] == [0, 1, 2, 3, 4]
    for x, s in zip(lines, st):
        assert tuple(x["sweeps"]) == s.sweeps and x["rhs"][0] == pytest.approx(s.rhs[0], rel=1e-15)
        assert x["n"] == [200, 136, 1] and x["tol"] == 1e-10
    assert all(x["sweeps"][0] > 0 and x["nonconverged"] == [0, 0] for x in lines)
