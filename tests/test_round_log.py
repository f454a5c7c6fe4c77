"""The per-round JSON-lines log of a plan (host logic, no GPU)."""
import io
import json

import numpy as np

from paper_1003_5402_amd.binding import write_round_log


def _plan():
    return dict(rounds=3, round_beam=np.array([2, 0, 2, 9], np.int32), round_rc=np.array([-3.0, -1.5, -0.25, 0.0]),
                round_gap=np.array([0.5, 1e-3, 2e-9, 0.0]), round_F=np.array([9.0, 7.5, 7.25, 0.0]),
                round_steps=np.array([1, 14, 500, 0], np.int32), round_kkt=np.array([0.0, 1e-9, 3e-6, 0.0]),
                round_stop=np.array([3, 1, 2, 0], np.int32))


def test_one_line_per_round_in_order(tmp_path):
    path = tmp_path / "plan.jsonl"
    assert write_round_log(_plan(), str(path), plan_id=7) == 3
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    assert [r["round"] for r in recs] == [0, 1, 2]
    assert [r["beam"] for r in recs] == [2, 0, 2]
    assert [r["stop"] for r in recs] == ["zero_direction", "kkt", "step_cap"]
    assert recs[2]["steps"] == 500 and recs[2]["kkt"] == 3e-6 and recs[1]["gap"] == 1e-3
    assert all(r["plan_id"] == 7 for r in recs)
    # appends: a second plan goes after the first
    write_round_log(_plan(), str(path), plan_id=8)
    assert len(path.read_text().splitlines()) == 6


def test_text_file_and_empty_plan():
    buf = io.StringIO()
    p = _plan()
    p["rounds"] = 0
    assert write_round_log(p, buf) == 0
    assert buf.getvalue() == ""
