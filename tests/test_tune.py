"""Host logic of the autotuner: order ranges from the measured orders, the
fastest setting per order and precision, and applying a stored table."""
import json

from paper_2312_13051_amd import _lib as L
from paper_2312_13051_amd import tune


class FakeCtx:
    def __init__(self):
        self.calls = []
        self.default = 512
        self.loads = 0

    def tune_clear(self, knob):
        self.calls.append(("clear", knob))

    def tune_set(self, knob, value):
        if knob == "hetrd_panel_loads":
            self.loads = value
        else:
            self.default = value

    def tune_set_orders(self, knob, n_lo, n_hi, precision, value):
        self.calls.append((knob, n_lo, n_hi, precision, value))


def test_autotune_picks_fastest_and_splits_orders(monkeypatch):
    # synthetic timings: 256 threads fastest below N = 300, 1024 above 1000, else 512
    def fake_time(ctx, N, precision, n_mat, reps=2, seed=0):
        want = 256 if N < 300 else (1024 if N > 1000 else 512)
        return 1.0 if ctx.default == want else 2.0 + ctx.default * 1e-4

    monkeypatch.setattr(tune, "time_eigh", fake_time)
    ctx = FakeCtx()
    table = tune.autotune(ctx, [2304, 128, 400], precisions=("mixed", "fp64"), log=lambda s: None)
    rows = table["knobs"]["hetrd_panel_threads"]
    assert [(r["n_lo"], r["n_hi"]) for r in rows[:3]] == [(1, 264), (265, 1352), (1353, (1 << 30) - 1)]
    assert [r["value"] for r in rows] == [256, 512, 1024] * 2
    assert [r["precision"] for r in rows] == [L.BE_MIXED_FP32] * 3 + [L.BE_FP64] * 3
    assert len(table["measurements"]) == 6 and table["measurements"][0]["best"] == "256"
    assert table["measurements"][1]["best"] == "512x4"
    # the loads knob: mixed-path rows only (the FP64 kernels have one form each)
    assert [r["precision"] for r in table["knobs"]["hetrd_panel_loads"]] == [L.BE_MIXED_FP32] * 3
    assert set(table["measurements"][0]["seconds"]) == {"256", "512x4", "512x8", "1024"}
    assert set(table["measurements"][3]["seconds"]) == {"256", "512", "1024"}


def test_autotune_picks_the_faster_load_form(monkeypatch):
    # 8 loads in flight faster from N = 1000 on; 512 threads fastest everywhere
    def fake_time(ctx, N, precision, n_mat, reps=2, seed=0):
        if ctx.default != 512:
            return 5.0
        if precision == L.BE_FP64:
            return 1.0
        return 1.0 if ctx.loads == (8 if N >= 1000 else 4) else 1.5

    monkeypatch.setattr(tune, "time_eigh", fake_time)
    table = tune.autotune(FakeCtx(), [400, 1024, 2304], precisions=("mixed", "fp64"), log=lambda s: None)
    assert [r["value"] for r in table["knobs"]["hetrd_panel_loads"]] == [4, 8, 8]
    assert [r["value"] for r in table["knobs"]["hetrd_panel_threads"]] == [512] * 6
    assert [m["best"] for m in table["measurements"]] == ["512x4", "512x8", "512x8", "512", "512", "512"]


def test_load_tuning_applies_rows_in_order(tmp_path):
    table = {"knobs": {"hetrd_panel_threads": [
        {"n_lo": 1, "n_hi": 300, "precision": 1, "value": 256},
        {"n_lo": 301, "n_hi": 5000, "precision": -1, "value": 1024}]}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(table))
    ctx = FakeCtx()
    out = L.Context.load_tuning(ctx, str(p))
    assert out == table
    assert ctx.calls == [("clear", "hetrd_panel_threads"), ("hetrd_panel_threads", 1, 300, 1, 256),
                         ("hetrd_panel_threads", 301, 5000, -1, 1024)]


def test_batch_sizes_bounded():
    assert tune.batch_for(16) == 1536
    assert tune.batch_for(1024) == 384
    assert tune.batch_for(2304) == 256          # one matrix per compute unit
    assert tune.batch_for(2304, n_cu=80) == 80
    assert tune.batch_for(8000) == 32
